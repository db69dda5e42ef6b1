// Internal declarations of the gfx950 formal-solution library: grid and
// context state, per-(ray, site) sweep records, and the host-side launchers
// that each kernel file exports.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <set>
#include <memory>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/vrt.h"

namespace vrt {

// An error carrying a status code; caught at the C ABI boundary.
struct Error : std::runtime_error {
  vrt_status code;
  Error(vrt_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

// Blocks of a one-dimensional grid covering `work` threads. One dispatch
// counts its work-items in 32 bits, so a larger launch is an error here
// instead of a silently truncated grid.
inline unsigned grid_blocks(int64_t work, int threads) {
  const int64_t b = (work + threads - 1) / threads;
  if (b * (int64_t)threads > (int64_t)0xffffffffLL)
    throw Error(VRT_E_ARG, "a launch of " + std::to_string(b * (int64_t)threads) +
                               " work-items exceeds the 2^32 of one dispatch");
  return (unsigned)b;
}

#define VRT_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::vrt::Error(VRT_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Floating-point part of one sweep record. The integer part is an int4:
// x = site, y = first upwind site (-1 at boundary sites), z = second upwind
// site (-1 if none), w = 2 * ray + (1 if the ray points up).
struct RecF32 {
  float w1, ds1, ds2, pad;
};
struct RecF64 {
  double w1, ds1, ds2, pad;
};

template <typename T> struct RecOf;
template <> struct RecOf<float> { using type = RecF32; };
template <> struct RecOf<double> { using type = RecF64; };

// Device buffer with RAII release.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t b) {
    if (b <= bytes && p) return;
    release();
    if (b == 0) b = 16;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error(VRT_E_NOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed: " + hipGetErrorString(e));
    }
    bytes = b;
  }
  template <typename T> T *as() const { return static_cast<T *>(p); }
};

// accelerator dies (XCDs) of the GPU; workgroups are dealt to them round-robin
constexpr int kDies = 8;

// lanes per record for m lane-vectors per row: the smallest power of two >= m, at most 64
inline int lanes_per_record(int32_t m) {
  if (m >= 33) return 64;
  if (m >= 17) return 32;
  if (m >= 9) return 16;
  if (m >= 5) return 8;
  if (m >= 3) return 4;
  if (m == 2) return 2;
  return 1;
}

// Wave items of the persistent sweep for one records-per-wave width: item i
// covers records [rec[i], rec[i] + cnt[i]) inside one level step.
struct PersistItems {
  int32_t spw = 0;
  int64_t n_items = 0;
  DevBuf rec, cnt;
};



}  // namespace vrt

struct vrt_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t capture_stream = nullptr;
  std::string err;

  // kernel timing (eager launches only)
  struct Timed {
    int kernel;
    hipEvent_t start, stop;
    int64_t units;
  };
  bool profiling = false;
  std::vector<Timed> pending;
  double prof_ms[3] = {0, 0, 0};
  int64_t prof_launches[3] = {0, 0, 0};
  int64_t prof_units[3] = {0, 0, 0};
  void drain_profile();

  // auxiliary streams (default priority) for sweeps split into independent
  // chains of rays, with the events that fork them from and join them to
  // the context stream
  std::vector<hipStream_t> aux;
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> join_ev;
  void ensure_aux(int k);

  // live grids of this context, destroyed with it
  std::set<vrt_grid_s *> grids;
};

struct vrt_grid_s {
  vrt_ctx ctx = nullptr;
  int kind = 0;  // 0 Voronoi, 1 regular
  int64_t n = 0;

  // Voronoi geometry
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  bool periodic = false;
  int64_t m = 0;
  vrt::DevBuf d_xyz, d_ptr, d_idx, d_shift, d_wall;
  std::vector<uint8_t> h_wall;
  std::vector<double> h_xyz;

  // regular geometry
  int32_t nx = 0, ny = 0, nz = 0;
  double dx = 0, dy = 0;
  std::vector<double> h_z;
  vrt::DevBuf d_z;

  // quadrature
  int32_t R = 0;
  std::vector<double> h_dirs, h_w;
  double r_exp = 7.0;
  vrt::DevBuf d_dirs, d_w;

  // Voronoi selection and schedule, [R][n] in caller site order
  vrt::DevBuf d_k1, d_k2, d_w1, d_ds1, d_ds2, d_level, d_order;
  std::vector<int32_t> n_levels;               // per ray
  std::vector<std::vector<int32_t>> level_ptr;  // per ray, [n_levels + 1]
  int64_t n_fallback = 0;

  // sweep records in step-major order: step s holds level s of ray 0, 1, ...
  int32_t n_steps = 0;
  int64_t n_rec = 0;
  vrt::DevBuf d_ri, d_rf32, d_rf64;
  std::vector<int64_t> step_ptr;  // [n_steps + 1]
  std::vector<int64_t> seg_off;   // [n_steps][R]: first record of (step, ray)
  std::vector<int64_t> seg_cnt;   // [n_steps][R]

  // emergent index
  std::vector<int64_t> em_off;
  std::vector<int32_t> em_site;
  vrt::DevBuf d_em_ray, d_em_site;

  // wavelength table of the LTE helper
  std::vector<double> h_lam;
  vrt::DevBuf d_lam;

  // tuning knobs
  int record_order = 1;  // 0 site index, 1 Morton (x, y) within a level
  int shared_levels = 0;  // 1: one level schedule per (hemisphere, azimuth) group of rays
  int xcd_chunks = 8;    // 0 = plain block order
  int ray_affinity = 0;  // 1: each ray's records always run on the same die
  int chains = 1;        // independent launch chains (streams) a sweep is split into
  int lane_bytes = 16;   // bytes of a row each lane moves per access (16 or 32)
  int ray_groups = 1;    // the rays are swept in this many consecutive passes
  int interleave = 0;    // step-wide sweeps read a copy of the records ordered across rays by the site's
                         // horizontal Morton code (1) or by site index (2); 0 = per-ray order
  int pipe = 0;          // > 0: level-step sweeps use the pipelined kernel with this many record groups per wave
  int regular_tiled = 2;  // regular grids: LDS-tiled plane kernel (1), row kernel (0), tiled in FP64 only (2)
  int segment = 0;       // 0: linear source along a line, 1: quadratic Bezier (needs the downwind lines)
  int reverse_persistent = 0;  // 1: the reverse sweep of a ray group runs as one persistent launch
  std::map<int64_t, std::unique_ptr<vrt::PersistItems>> reverse_items;  // keyed by (spw, first ray, group)
  vrt::DevBuf d_q1, d_q2, d_qw1, d_qd1, d_qd2;  // downwind lines [R][n]: the selection of the opposite rays
  bool down_built = false;
  vrt::DevBuf d_ri_x, d_rf32_x, d_rf64_x;
  int interleaved_built = 0;  // interleave mode of the copy in d_ri_x, d_rf*_x (0 = none)
  int tuned_exec = VRT_EXEC_GRAPH;  // launch mode chosen by the autotuner (VRT_EXEC_AUTO resolves to it)

  // ray-affinity tables: ray_die[r], and per step [kDies][xk][2] = {first
  // record, running count} over the segments of each die's rays
  std::vector<int32_t> ray_die;
  int32_t xk = 0;
  std::vector<int64_t> xmax;  // [n_steps]: largest record count of one die
  vrt::DevBuf d_xtab;

  // scratch for per-ray intensities when the caller passes none
  vrt::DevBuf d_Iscr;
  const void *last_I = nullptr;  // intensities of the last solution (library scratch)
  bool last_abs = false;         // last_I holds sign-encoded rows (read as |I|)
  // rows of the sign-encoded persistent sweep, owned by that mode alone, and the
  // layout {element bytes, wavelengths, rays, sites} they were last filled for
  vrt::DevBuf d_Isgn;
  int64_t sgn_key[4] = {0, 0, 0, 0};
  int last_prec = -1;            // their precision, wavelength count and row stride
  int32_t last_nl = 0, last_ld = 0;
  bool last_own = false;         // last_I is one of the library's own row blocks
  // identifies the last solution whose rows last_I holds: it grows with every
  // call that writes or drops the library's rows (or finds a device error)
  int64_t solution_id = 0;

  // persistent sweep state: per-(ray, site) epoch stamps, the epoch, a device
  // error flag (a bounded wait gave up) and wave-item tables by width
  vrt::DevBuf d_flags, d_epoch;
  std::map<int32_t, std::unique_ptr<vrt::PersistItems>> persist_items;
  int32_t persist_max_blocks = 0;  // persistent-sweep workgroups; 0 = as many as can be resident
  int64_t spin_cap = int64_t(1) << 22;

  // two-level iteration scratch: chi, S, I_bottom in the sweep precision, the
  // profile weights, the max-change word and its pinned host copy
  vrt::DevBuf d_nchi, d_nIb, d_wlam, d_dS, d_atm_ptr, d_active, d_jbar, d_lbar;
  unsigned long long *h_dS = nullptr;  // pinned, [n_atm]
  int32_t *h_active = nullptr;         // pinned, [n_atm]
  int32_t h_dS_cap = 0;
  hipGraphExec_t nlte_graph = nullptr;
  std::tuple<int, int32_t, const void *, const void *, const void *, const void *, const void *, double, int, int32_t,
             const void *, const void *, const void *, int>
      nlte_key{};
  const void *nlte_scratch[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};

  // reverse sweep: per-ray dependents lists (absolute offsets [R][n+1], the
  // dependent site, and the weight and length of the line it reads), scratch
  vrt::DevBuf d_dep_ptr, d_dep_site, d_dep_rf32, d_dep_rf64;
  bool deps_built = false;
  vrt::DevBuf d_vI, d_vIbar, d_vSbar, d_vCbar, d_vacc;
  // checkpointed forward intensities of the reverse sweep: per record
  // {chunk slot, frontier slot or -1, upwind row locations} for level chunks
  // of ck_levels steps and ray groups of ck_group rays (0 = not built), the
  // row counts of the chunk and frontier buffers, and the buffers
  vrt::DevBuf d_ck, d_vIch, d_vIfr;
  int32_t ck_levels = 0, ck_group = 0;
  int64_t ck_chunk_rows = 0, ck_front_rows = 0;

  // final synthesis on a regular grid: per-point packed line data and the
  // nearest-site walk's error flag
  vrt::DevBuf d_pack, d_walk_bad, d_brute;

  // captured launch sequences, keyed by (prec, n_lambda, chi / S row stride, pointers)
  using GraphKey =
      std::tuple<int, int32_t, int64_t, const void *, const void *, const void *, const void *, void *, void *>;
  std::map<GraphKey, hipGraphExec_t> graphs;
  void drop_graphs();
};

namespace vrt {

// ---- k_select.hip
void launch_select(hipStream_t s, int64_t n, int32_t R, const double *xyz, const int64_t *ptr,
                   const int32_t *idx, const int8_t *shift, const uint8_t *wall, double Lx, double Ly,
                   const double *dirs, double r_exp, int32_t *k1, int32_t *k2, double *w1, double *ds1,
                   double *ds2, unsigned long long *n_fallback, int32_t *bad_site);

// ---- k_schedule.hip
void launch_level_fill(hipStream_t s, int64_t total, int32_t *level);
void launch_level_relax(hipStream_t s, int64_t n, int32_t R, const int32_t *k1, const int32_t *k2,
                        int32_t *level, int32_t *changed, const int32_t *peer = nullptr, int32_t P = 0);
void launch_level_count(hipStream_t s, int64_t n, int32_t R, int32_t Lmax, int64_t tile,
                        const int32_t *level, int32_t *cnt, const int32_t *visit);
void launch_level_scan(hipStream_t s, int32_t R, int32_t Lmax, int64_t ntiles, int32_t *cnt,
                       int64_t *totals);
void launch_level_ptr(hipStream_t s, int32_t R, int32_t Lmax, const int64_t *totals, int32_t *level_ptr,
                      int32_t *n_levels);
void launch_level_scatter(hipStream_t s, int64_t n, int32_t R, int32_t Lmax, int64_t tile,
                          const int32_t *level, const int32_t *level_ptr, int32_t *cnt, int32_t *order,
                          const int32_t *visit);
void launch_level_max(hipStream_t s, int64_t total, const int32_t *level, int32_t *out_max);
void launch_pack(hipStream_t s, int64_t n, int32_t R, int32_t Lmax, const int32_t *order,
                 const int32_t *level, const int32_t *level_ptr, const int64_t *seg_off,
                 const int32_t *k1, const int32_t *k2, const double *w1, const double *ds1,
                 const double *ds2, const double *dirs, int4 *ri, RecF32 *rf32, RecF64 *rf64);

// ---- k_sweep.hip
// I holds the rays from ray0 on (ray r writes I + (r - ray0) * n * nl). With
// xtab (one step's ray-affinity table [kDies][xk][2]), rec_count is the
// largest record count of one die and rec_begin is unused. pipe > 0: each
// wavefront sweeps pipe (2, 4 or 8) groups of records with the next groups'
// loads in flight (16-byte lanes, rows of at most one lane-vector per lane,
// ray0 = 0, no affinity table; otherwise the classic kernel runs). The
// pipelined kernel updates interior records only: pass pipe > 0 for level
// steps >= 1 (step 0 holds exactly the boundary sites).
// The input rows of site i (chi, S, Ibot, Itop) start at i cs (cs >= nl; cs =
// nl for arrays of n x nl); intensity rows are nl apart.
template <typename T>
void launch_sweep(hipStream_t s, const int4 *ri, const typename RecOf<T>::type *rf, int64_t rec_begin,
                  int64_t rec_count, int32_t nl, int64_t cs, int64_t n, const T *chi, const T *S, const T *Ibot,
                  const T *Itop, T *I, int32_t xcd_chunks, int32_t ray0, const int64_t *xtab = nullptr,
                  int32_t xk = 0, int32_t lane_bytes = 16, int32_t pipe = 0);
// Forward sweep of records [rec_begin, rec_begin + rec_count) with checkpointed
// rows: ck[rec] = {chunk slot, frontier slot or -1, upwind location of line 1,
// of line 2} (location >= 0: chunk slot in Ich; -(f + 1): frontier slot f in
// Ifr); rows of nl entries. Same arithmetic as launch_sweep.
template <typename T>
void launch_sweep_ck(hipStream_t s, const int4 *ri, const typename RecOf<T>::type *rf, const int4 *ck,
                     int64_t rec_begin, int64_t rec_count, int32_t nl, const T *chi, const T *S, const T *Ibot,
                     const T *Itop, T *Ich, T *Ifr);
// abs_rows: I holds sign-encoded rows (read as |I|); then err is the persistent
// sweep's device error word, and a set word makes the outputs NaN (the rows
// are not the current epoch's)
template <typename T>
void launch_jreduce(hipStream_t s, const T *I, int32_t R, int64_t nn, const double *w, T *J,
                    bool abs_rows = false, const int32_t *err = nullptr);
template <typename T>
void launch_emergent(hipStream_t s, int64_t total, int32_t nl, int32_t ld, int64_t n, const int32_t *em_ray,
                     const int32_t *em_site, const T *I, T *out, bool abs_rows = false,
                     const int32_t *err = nullptr);

// ---- k_source.hip
// rows of site i at i cs (cs >= nl)
template <typename T>
void launch_lte(hipStream_t s, int64_t n, int32_t nl, int64_t cs, const double *lam, double kappa0, const double *T_,
                const double *rho, T *chi, T *S);

// ---- k_persist.hip
// words: [0] epoch, [1] device error (non-zero: a bounded wait gave up),
// [2] registration word, [3] frozen wavefront count + 1. Flags of ray r start
// at flags + r * flag_ld.
// starts a persistent sweep: bumps the stamped (sign = false) or the sign-encoded
// (sign = true) epoch and resets the registration words
void launch_persist_begin(hipStream_t s, int32_t *words, bool sign = false);
// fills count elements with zeros of the current sign-encoded epoch's sign
template <typename T> void launch_sign_fill(hipStream_t s, T *p, int64_t count, const int32_t *words);
// records per wavefront of the persistent sweep for rows of nl entries and a
// chi / S row stride cs
int32_t persistent_records_per_wave(int32_t nl, int elem_bytes, bool aligned, int64_t cs);
bool al16(const void *p);
template <typename T>
void launch_persistent_sweep(hipStream_t s, const PersistItems &items, int32_t max_blocks, const int4 *ri,
                             const typename RecOf<T>::type *rf, int32_t nl, int64_t cs, int64_t n, int64_t flag_ld,
                             const T *chi, const T *S, const T *Ibot, const T *Itop, T *I, int32_t *flags,
                             int32_t *words, int64_t spin_cap, bool sign = false, int32_t mixed_rays = 0);

// dst[i] = |src[i]| (abs) or src[i], converted to T; NaN everywhere when the
// persistent sweeps' error word (err, may be null) is set
template <typename T>
void launch_rows_convert(hipStream_t s, const void *src, bool src_f32, bool abs, T *dst, int64_t count,
                         const int32_t *err);

// ---- k_nlte.hip
// rows of ld entries, cs apart
template <typename T>
void launch_nlte_assemble(hipStream_t s, int64_t n, int32_t nl, int32_t ld, int64_t cs, const double *phi,
                          const double *chi_L, const double *chi_c, const double *B, const double *S_L, T *chi,
                          T *S);
template <typename T>
void launch_broadcast(hipStream_t s, int64_t n, int32_t ld, int64_t cs, const double *v, T *out);
void launch_zero_u64(hipStream_t s, int32_t count, unsigned long long *p);
// sets *bad to 1 if a selected upwind neighbour of a site lies in another atmosphere
void launch_check_partition(hipStream_t s, int64_t n, int32_t R, const int32_t *k1, const int32_t *k2, int32_t n_atm,
                            const int64_t *atm_ptr, int32_t *bad);
template <typename T>
void launch_line_update(hipStream_t s, int64_t n, int32_t nl, int32_t ld, int32_t R, const T *I, const double *w,
                        const double *wlam, const double *phi, const double *B, double eps, double *S_L,
                        int32_t n_atm, const int64_t *atm_ptr, const int32_t *active, unsigned long long *dS_bits,
                        double *Jbar, const double *Lbar);
// diagonal of the line operator per site (accelerated iteration)
void launch_line_diag(hipStream_t s, int64_t n, int32_t nl, int32_t R, const double *ray_w, const int32_t *k1,
                      const int32_t *k2, const double *w1, const double *ds1, const double *ds2, const double *chi_c,
                      const double *chi_L, const double *phi, const double *wlam, double *Lbar);

// ---- k_adjoint.hip
template <typename T>
void launch_reverse(hipStream_t s, const int4 *ri, const typename RecOf<T>::type *rf, int64_t rec_begin,
                    int64_t rec_count, int32_t nl, int64_t n, int32_t ray0, const int64_t *dep_ptr,
                    const int32_t *dep_site, const typename RecOf<T>::type *dep_rec, const T *chi, const T *S,
                    const T *I, const T *gI, const T *gJ, const double *ray_w, T *Ibar, T *Sbar, T *Cbar,
                    const int4 *ck = nullptr, const T *Ich = nullptr, const T *Ifr = nullptr);
// Every level step of a ray group's reverse sweep in one launch; items from
// the group's (step, ray) segments in decreasing step order, item_cnt =
// count + 256 x (ray - ray0); stamps and words as for the persistent sweep.
int32_t reverse_records_per_wave(int32_t nl, int elem_bytes, bool aligned);
template <typename T>
void launch_persistent_reverse(hipStream_t s, const PersistItems &items, int32_t max_blocks, const int4 *ri,
                               const typename RecOf<T>::type *rf, int32_t nl, int64_t n, int32_t ray0,
                               const int64_t *dep_ptr, const int32_t *dep_site, const typename RecOf<T>::type *dep_rec,
                               const T *chi, const T *S, const T *I, const T *gI, const T *gJ, const double *ray_w,
                               T *Ibar, T *Sbar, T *Cbar, int64_t flag_ld, int32_t *flags, int32_t *words,
                               int64_t spin_cap);
template <typename T>
void launch_reverse_reduce(hipStream_t s, int64_t n, int32_t nl, int32_t ray0, int32_t group, const double *dirs,
                           const uint8_t *wall, const T *Ibar, const T *Sbar, const T *Cbar, double *acc_chi,
                           double *acc_S, double *acc_Ib, double *acc_It);
template <typename T> void launch_to_prec(hipStream_t s, int64_t nn, const double *a, T *out);
template <typename T> void launch_fill_zero(hipStream_t s, int64_t count, T *p);
template <typename T>
void launch_emergent_scatter(hipStream_t s, int64_t total, int32_t nl, int64_t n, const int32_t *em_ray,
                             const int32_t *em_site, const T *g_em, T *gI);
template <typename T>
void launch_lte_vjp(hipStream_t s, int64_t n, int32_t nl, const double *lam, double kappa0, const double *T_,
                    const double *rho, const T *g_chi, const T *g_S, const T *g_Ib, double *g_T, double *g_rho);

// ---- k_regular.hip
template <typename T>
void launch_regular(hipStream_t s, int32_t step, int32_t ray_begin, int32_t ray_count, int32_t nx,
                    int32_t ny, int32_t nz, double dx, double dy, const double *z, const double *dirs,
                    int32_t nl, const T *chi, const T *S, const T *Ibot, const T *Itop, T *I, bool tiled = true,
                    int32_t xcd_chunks = 8);

// ---- k_bezier.hip
// the quadratic Bezier sweep of a contiguous record range; q1, q2, qw1, qd1,
// qd2 [R][n] are the downwind lines (the upwind selection of the opposite rays)
// Every ray and level of the quadratic-segment sweep in one launch (items of
// bezier_records_per_wave() records; stamps and words as for the persistent
// linear sweep).
int32_t bezier_records_per_wave();
template <typename T>
void launch_persistent_bezier(hipStream_t s, const PersistItems &items, int32_t max_blocks, const int4 *ri,
                              const typename RecOf<T>::type *rf, int32_t nl, int64_t cs, int64_t n, const int32_t *q1,
                              const int32_t *q2, const double *qw1, const double *qd1, const double *qd2,
                              const T *chi, const T *S, const T *Ibot, const T *Itop, T *I, int64_t flag_ld,
                              int32_t *flags, int32_t *words, int64_t spin_cap);
template <typename T>
void launch_bezier_sweep(hipStream_t s, const int4 *ri, const typename RecOf<T>::type *rf, int64_t rec_begin,
                         int64_t rec_count, int32_t nl, int64_t cs, int64_t n, const int32_t *q1, const int32_t *q2,
                         const double *qw1, const double *qd1, const double *qd2, const T *chi, const T *S,
                         const T *Ibot, const T *Itop, T *I, int32_t xcd_chunks);

// ---- k_synth.hip
// the two nearest sites of the points on the lattice of one stride, by brute
// force over all sites (the coarsest level of the search); pb, pe hold
// idw_brute_scratch_pairs() pairs of (site, key)
int64_t idw_brute_scratch_pairs(int32_t nx, int32_t ny, int32_t nz, int32_t stride, int64_t n);
void launch_idw_brute(hipStream_t s, int32_t nx, int32_t ny, int32_t nz, double dx, double dy, const double *z,
                      int32_t stride, int64_t n, const double *xyz, bool periodic, double Lx, double Ly, double power,
                      int32_t *idx, double *w1, double *d2, int32_t *pb, double *pe);
// one finer level of the search: the points of lattice `stride` not on lattice
// `parent`, each walking from its parent point's nearest site
void launch_idw_level(hipStream_t s, int32_t nx, int32_t ny, int32_t nz, double dx, double dy, const double *z,
                      int32_t stride, int32_t parent, int64_t n, const double *xyz, const int64_t *ptr,
                      const int32_t *nbr, bool periodic, double Lx, double Ly, double power, int32_t *idx,
                      double *w1, double *d2, int32_t *bad);
void launch_idw_apply(hipStream_t s, int64_t m, int32_t nc, int64_t n_src, const int32_t *idx, const double *w1,
                      const double *src, double *dst);
// pack holds m float4 (T = float) or double4 (T = double)
template <typename T>
void launch_line_pack(hipStream_t s, int64_t m, int64_t n_src, const int32_t *idx, const double *w1,
                      const double *S_site, const double *chi_L, const double *chi_c, const double *B, void *pack);
template <typename T>
void launch_vertical_line(hipStream_t s, int64_t ncol, int32_t nz, int32_t nl, const double *z, const T *phi,
                          const void *pack, const double *B, const T *Ib, T *out);
template <typename T>
void launch_vertical_plain(hipStream_t s, int64_t ncol, int32_t nz, int32_t nl, const double *z, const T *chi,
                           const T *S, const T *Ib, T *out);

}  // namespace vrt
