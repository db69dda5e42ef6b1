// C ABI of the formal-solution library: contexts, grids, validation, the
// construction of per-ray sweep schedules on the GPU, and the launch
// sequences of the formal solution (plain, batched, or captured into a HIP
// graph). Every entry point converts internal errors into a status code and a
// message on the context; no exception crosses the ABI.

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <thread>

#include "vrt_internal.h"

using vrt::DevBuf;
using vrt::Error;

// Scratch of vrt_formal_solution_noalloc, the entry point that allocates
// nothing: the per-ray intensities live in this file-scope device array. Every
// GPU the library runs on holds its own copy until the process ends. In host
// code the name is not a device address: the address comes from
// hipGetSymbolAddress, once per device with that device current, when a
// context is created on it (scratch_dev below), and only that address is
// passed to kernels.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// records the device address of `scratch` on the current device (called with
// `device` current); returns false if the runtime cannot give it
bool init_scratch_dev(int device) {
  if (device < 0 || device >= kMaxDevices) return false;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device]) return true;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return false;
  g_scratch_dev[device] = p;
  return true;
}

void *scratch_dev(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_dev[device];
}

constexpr const char *kVersion = "vrt 0.1.0 (gfx950)";

template <typename F> vrt_status guarded(vrt_ctx ctx, F &&f) {
  try {
    if (ctx) {
      ctx->err.clear();
      VRT_HIP(hipSetDevice(ctx->device));
    }
    return f();
  } catch (const Error &e) {
    if (ctx) ctx->err = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    if (ctx) ctx->err = "host allocation failed";
    return VRT_E_NOMEM;
  } catch (const std::exception &e) {
    if (ctx) ctx->err = e.what();
    return VRT_E_HIP;
  }
}

void fail(vrt_status code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void fail(vrt_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  throw Error(code, buf);
}

template <typename T> void upload(DevBuf &d, const T *h, size_t count, hipStream_t s) {
  d.alloc(count * sizeof(T));
  if (count) VRT_HIP(hipMemcpyAsync(d.p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
}

// Host-side geometry checks (reading of Sect. 2.4: a Voronoi diagram's
// neighbour relation is symmetric and each shared face is one entry on each
// side). Returns an empty string when the grid is well formed.
std::string check_voronoi(int64_t n, const double *xyz, const int64_t *ptr, const int32_t *idx, const int8_t *shift,
                          const uint8_t *wall, const double lo[3], const double hi[3], bool periodic) {
  char buf[256];
  if (n < 0) return "negative site count";
  if (n > 0 && (!xyz || !ptr || !wall)) return "null xyz, nbr_ptr or wall";
  if (n >= (int64_t(1) << 31)) return "more than 2^31 - 1 sites";
  if (ptr && ptr[0] != 0) return "nbr_ptr[0] must be 0";
  for (int d = 0; d < 3; ++d)
    if (!(hi[d] > lo[d])) return "box must satisfy hi > lo in every dimension";
  int64_t m = n > 0 ? ptr[n] : 0;
  if (m > 0 && !idx) return "null nbr_idx";
  if (periodic && m > 0 && !shift) return "periodic grid needs nbr_shift";
  for (int64_t i = 0; i < n; ++i) {
    if (ptr[i + 1] < ptr[i]) {
      snprintf(buf, sizeof buf, "nbr_ptr decreases at site %lld", (long long)i);
      return buf;
    }
    if (wall[i] & ~3u) {
      snprintf(buf, sizeof buf, "wall flag of site %lld uses bits other than 0 and 1", (long long)i);
      return buf;
    }
    for (int d = 0; d < 3; ++d) {
      const double v = xyz[3 * i + d];
      if (!std::isfinite(v) || v < lo[d] || v > hi[d]) {
        snprintf(buf, sizeof buf, "site %lld lies outside the box", (long long)i);
        return buf;
      }
    }
  }
  // per-row sorted copies of (k, sx, sy) to look up reverse entries
  struct Ent {
    int32_t k;
    int8_t sx, sy;
    bool operator<(const Ent &o) const { return std::tie(k, sx, sy) < std::tie(o.k, o.sx, o.sy); }
    bool operator==(const Ent &o) const { return k == o.k && sx == o.sx && sy == o.sy; }
  };
  std::vector<Ent> ent((size_t)m);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
      const int32_t k = idx[e];
      const int8_t sx = shift ? shift[2 * e] : 0, sy = shift ? shift[2 * e + 1] : 0;
      if (k < 0 || k >= n) {
        snprintf(buf, sizeof buf, "neighbour index %d of site %lld out of range", k, (long long)i);
        return buf;
      }
      if (sx < -1 || sx > 1 || sy < -1 || sy > 1) {
        snprintf(buf, sizeof buf, "shift of entry %lld not in {-1,0,1}", (long long)e);
        return buf;
      }
      if (!periodic && (sx || sy)) {
        snprintf(buf, sizeof buf, "non-zero shift on a non-periodic grid (entry %lld)", (long long)e);
        return buf;
      }
      if (k == i && sx == 0 && sy == 0) {
        snprintf(buf, sizeof buf, "site %lld lists itself without a periodic shift", (long long)i);
        return buf;
      }
      ent[(size_t)e] = Ent{k, sx, sy};
    }
    std::sort(ent.begin() + ptr[i], ent.begin() + ptr[i + 1]);
    if (std::adjacent_find(ent.begin() + ptr[i], ent.begin() + ptr[i + 1]) != ent.begin() + ptr[i + 1]) {
      snprintf(buf, sizeof buf, "site %lld lists a neighbour twice", (long long)i);
      return buf;
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
      const Ent rev{(int32_t)i, (int8_t)-ent[(size_t)e].sx, (int8_t)-ent[(size_t)e].sy};
      const int32_t k = ent[(size_t)e].k;
      if (!std::binary_search(ent.begin() + ptr[k], ent.begin() + ptr[k + 1], rev)) {
        snprintf(buf, sizeof buf, "neighbour lists are not symmetric: %lld lists %d but not the reverse",
                 (long long)i, k);
        return buf;
      }
    }
  }
  return "";
}

template <typename T> const typename vrt::RecOf<T>::type *records(vrt_grid g);
template <> const vrt::RecF32 *records<float>(vrt_grid g) { return g->d_rf32.as<vrt::RecF32>(); }
template <> const vrt::RecF64 *records<double>(vrt_grid g) { return g->d_rf64.as<vrt::RecF64>(); }

void build_emergent_index(vrt_grid g) {
  g->em_off.assign((size_t)g->R + 1, 0);
  g->em_site.clear();
  std::vector<int32_t> ray_of;
  for (int32_t r = 0; r < g->R; ++r) {
    const bool up = g->h_dirs[3 * r + 2] > 0.0;
    if (g->kind == 0) {
      const uint8_t bit = up ? 2 : 1;  // downwind wall
      for (int64_t i = 0; i < g->n; ++i)
        if (g->h_wall[(size_t)i] & bit) {
          g->em_site.push_back((int32_t)i);
          ray_of.push_back(r);
        }
    } else {
      const int64_t plane = (int64_t)g->nx * g->ny;
      const int64_t k = up ? g->nz - 1 : 0;
      for (int64_t p = 0; p < plane; ++p) {
        g->em_site.push_back((int32_t)(k * plane + p));
        ray_of.push_back(r);
      }
    }
    g->em_off[(size_t)r + 1] = (int64_t)g->em_site.size();
  }
  upload(g->d_em_site, g->em_site.data(), g->em_site.size(), g->ctx->stream);
  upload(g->d_em_ray, ray_of.data(), ray_of.size(), g->ctx->stream);
  VRT_HIP(hipStreamSynchronize(g->ctx->stream));
}

// Ray-affinity tables: rays sorted by their number of levels (most first, then
// index) are dealt to the dies in serpentine order, so every die gets a mix of
// long and short sweeps; per step, each die's records are the (level, ray)
// segments of its rays.
void build_affinity(vrt_grid g) {
  const int32_t R = g->R, NS = g->n_steps, D = vrt::kDies;
  std::vector<int32_t> by((size_t)R);
  for (int32_t r = 0; r < R; ++r) by[(size_t)r] = r;
  std::stable_sort(by.begin(), by.end(),
                   [&](int32_t a, int32_t b) { return g->n_levels[(size_t)a] > g->n_levels[(size_t)b]; });
  g->ray_die.assign((size_t)R, 0);
  std::vector<std::vector<int32_t>> rays_of((size_t)D);
  for (int32_t p = 0; p < R; ++p) {
    const int32_t round = p / D, pos = p % D;
    const int32_t die = (round % 2 == 0) ? pos : D - 1 - pos;
    g->ray_die[(size_t)by[(size_t)p]] = die;
  }
  for (int32_t r = 0; r < R; ++r) rays_of[(size_t)g->ray_die[(size_t)r]].push_back(r);
  int32_t xk = 1;
  for (const auto &v : rays_of) xk = std::max<int32_t>(xk, (int32_t)v.size());
  g->xk = xk;
  std::vector<int64_t> tab((size_t)std::max(NS, 1) * D * xk * 2, 0);
  g->xmax.assign((size_t)NS, 0);
  for (int32_t st = 0; st < NS; ++st) {
    for (int32_t x = 0; x < D; ++x) {
      int64_t *t = tab.data() + ((size_t)st * D + x) * xk * 2;
      int64_t cum = 0;
      const auto &v = rays_of[(size_t)x];
      for (int32_t k = 0; k < xk; ++k) {
        if (k < (int32_t)v.size()) {
          const int32_t r = v[(size_t)k];
          t[2 * k] = g->seg_off[(size_t)st * R + r];
          cum += g->seg_cnt[(size_t)st * R + r];
        }
        t[2 * k + 1] = cum;  // unused slots repeat the total
      }
      g->xmax[(size_t)st] = std::max(g->xmax[(size_t)st], cum);
    }
  }
  upload(g->d_xtab, tab.data(), tab.size(), g->ctx->stream);
  VRT_HIP(hipStreamSynchronize(g->ctx->stream));  // the host table is local
}


// Morton code of each site's horizontal position in the box (16 bits per axis)
std::vector<uint64_t> morton_codes(vrt_grid g) {
  const int64_t n = g->n;
  std::vector<uint64_t> code((size_t)n);
  const std::vector<double> &xyz = g->h_xyz;
  const double Lx = g->hi[0] - g->lo[0], Ly = g->hi[1] - g->lo[1];
  auto q = [](double v) {
    double f = std::floor(v * 65536.0);
    return (uint32_t)std::min(65535.0, std::max(0.0, f));
  };
  for (int64_t i = 0; i < n; ++i) {
    const uint32_t ux = q((xyz[3 * i] - g->lo[0]) / Lx), uy = q((xyz[3 * i + 1] - g->lo[1]) / Ly);
    uint64_t m = 0;
    for (int b = 0; b < 16; ++b) m |= (uint64_t)((ux >> b) & 1u) << (2 * b) | (uint64_t)((uy >> b) & 1u) << (2 * b + 1);
    code[(size_t)i] = m;
  }
  return code;
}

// The records of every level step reordered across rays: by (Morton code of
// the site, ray, site) for interleave mode 1, by (site, ray) for mode 2 (with
// sites numbered along space, as a batch of atmospheres is, this keeps each
// atmosphere's records together). The records of one step are independent,
// so any order within a step gives the same intensities.
void build_interleaved(vrt_grid g) {
  hipStream_t s = g->ctx->stream;
  const int64_t nr = g->n_rec;
  std::vector<int4> ri((size_t)nr);
  std::vector<vrt::RecF32> r32((size_t)nr);
  std::vector<vrt::RecF64> r64((size_t)nr);
  VRT_HIP(hipMemcpyAsync(ri.data(), g->d_ri.p, (size_t)nr * sizeof(int4), hipMemcpyDeviceToHost, s));
  VRT_HIP(hipMemcpyAsync(r32.data(), g->d_rf32.p, (size_t)nr * sizeof(vrt::RecF32), hipMemcpyDeviceToHost, s));
  VRT_HIP(hipMemcpyAsync(r64.data(), g->d_rf64.p, (size_t)nr * sizeof(vrt::RecF64), hipMemcpyDeviceToHost, s));
  VRT_HIP(hipStreamSynchronize(s));
  const bool by_site = g->interleave == 2;
  const std::vector<uint64_t> code = by_site ? std::vector<uint64_t>() : morton_codes(g);
  std::vector<int64_t> perm((size_t)nr);
  std::iota(perm.begin(), perm.end(), int64_t(0));
  std::vector<int4> ri2((size_t)nr);
  std::vector<vrt::RecF32> r32b((size_t)nr);
  std::vector<vrt::RecF64> r64b((size_t)nr);
  // steps are independent: host threads take every nth step
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  auto work = [&](int t) {
    for (int32_t st = t; st < g->n_steps; st += nth) {
      const int64_t b0 = g->step_ptr[(size_t)st], e0 = g->step_ptr[(size_t)st + 1];
      std::sort(perm.begin() + b0, perm.begin() + e0, [&](int64_t u, int64_t v) {
        const int4 &a = ri[(size_t)u], &c = ri[(size_t)v];
        const uint64_t ka = by_site ? (uint64_t)a.x : code[(size_t)a.x];
        const uint64_t kc = by_site ? (uint64_t)c.x : code[(size_t)c.x];
        if (ka != kc) return ka < kc;
        if (a.w != c.w) return a.w < c.w;
        return a.x < c.x;
      });
      for (int64_t k = b0; k < e0; ++k) {
        ri2[(size_t)k] = ri[(size_t)perm[(size_t)k]];
        r32b[(size_t)k] = r32[(size_t)perm[(size_t)k]];
        r64b[(size_t)k] = r64[(size_t)perm[(size_t)k]];
      }
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nth; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto &th : pool) th.join();
  upload(g->d_ri_x, ri2.data(), ri2.size(), s);
  upload(g->d_rf32_x, r32b.data(), r32b.size(), s);
  upload(g->d_rf64_x, r64b.data(), r64b.size(), s);
  VRT_HIP(hipStreamSynchronize(s));  // the host vectors must outlive the copies
  g->interleaved_built = g->interleave;
}

// Downwind lines of every (ray, site) for the quadratic segment: the upwind
// selection (Eq. 5-6, the same rules) for the opposite direction.
void build_downwind(vrt_grid g) {
  hipStream_t s = g->ctx->stream;
  const int64_t n = g->n;
  const int32_t R = g->R;
  const int64_t RN = (int64_t)R * n;
  std::vector<double> neg(g->h_dirs.size());
  for (size_t k = 0; k < neg.size(); ++k) neg[k] = -g->h_dirs[k];
  DevBuf d_neg, d_misc;
  upload(d_neg, neg.data(), neg.size(), s);
  g->d_q1.alloc(RN * 4);
  g->d_q2.alloc(RN * 4);
  g->d_qw1.alloc(RN * 8);
  g->d_qd1.alloc(RN * 8);
  g->d_qd2.alloc(RN * 8);
  d_misc.alloc(sizeof(unsigned long long) * (size_t)R + 16);
  auto *d_nfb = d_misc.as<unsigned long long>();
  auto *d_bad = reinterpret_cast<int32_t *>(d_nfb + R);
  VRT_HIP(hipMemsetAsync(d_nfb, 0, sizeof(unsigned long long) * (size_t)R, s));
  const int32_t big = 0x7fffffff;
  VRT_HIP(hipMemcpyAsync(d_bad, &big, 4, hipMemcpyHostToDevice, s));
  const double Lx = g->periodic ? g->hi[0] - g->lo[0] : 0.0;
  const double Ly = g->periodic ? g->hi[1] - g->lo[1] : 0.0;
  vrt::launch_select(s, n, R, g->d_xyz.as<double>(), g->d_ptr.as<int64_t>(), g->d_idx.as<int32_t>(),
                     g->d_shift.as<int8_t>(), g->d_wall.as<uint8_t>(), Lx, Ly, d_neg.as<double>(), g->r_exp,
                     g->d_q1.as<int32_t>(), g->d_q2.as<int32_t>(), g->d_qw1.as<double>(), g->d_qd1.as<double>(),
                     g->d_qd2.as<double>(), d_nfb, d_bad);
  int32_t bad = 0;
  VRT_HIP(hipMemcpyAsync(&bad, d_bad, 4, hipMemcpyDeviceToHost, s));
  VRT_HIP(hipStreamSynchronize(s));  // the host direction table must outlive the copy
  if (bad != big) fail(VRT_E_GRID, "site %d has no neighbour downwind in height", bad);
  g->down_built = true;
}

void set_rays_voronoi(vrt_grid g) {
  hipStream_t s = g->ctx->stream;
  const int64_t n = g->n;
  const int32_t R = g->R;
  const int64_t RN = (int64_t)R * n;
  // the wave-item tables and captured launches follow the level steps
  g->drop_graphs();
  g->persist_items.clear();
  g->reverse_items.clear();
  g->d_k1.alloc(RN * 4);
  g->d_k2.alloc(RN * 4);
  g->d_w1.alloc(RN * 8);
  g->d_ds1.alloc(RN * 8);
  g->d_ds2.alloc(RN * 8);
  g->d_level.alloc(RN * 4);
  g->d_order.alloc(RN * 4);

  // upwind selection (Eq. 5-6)
  DevBuf d_misc;
  d_misc.alloc(sizeof(unsigned long long) * (size_t)R + 64 + 4 * 16);
  auto *d_nfb = d_misc.as<unsigned long long>();
  auto *d_bad = reinterpret_cast<int32_t *>(d_nfb + R);
  auto *d_flags = d_bad + 4;  // 16 relaxation flags
  VRT_HIP(hipMemsetAsync(d_nfb, 0, sizeof(unsigned long long) * (size_t)R, s));
  const int32_t big = 0x7fffffff;
  VRT_HIP(hipMemcpyAsync(d_bad, &big, 4, hipMemcpyHostToDevice, s));
  const double Lx = g->periodic ? g->hi[0] - g->lo[0] : 0.0;
  const double Ly = g->periodic ? g->hi[1] - g->lo[1] : 0.0;
  vrt::launch_select(s, n, R, g->d_xyz.as<double>(), g->d_ptr.as<int64_t>(), g->d_idx.as<int32_t>(),
                     g->d_shift.as<int8_t>(), g->d_wall.as<uint8_t>(), Lx, Ly, g->d_dirs.as<double>(), g->r_exp,
                     g->d_k1.as<int32_t>(), g->d_k2.as<int32_t>(), g->d_w1.as<double>(), g->d_ds1.as<double>(),
                     g->d_ds2.as<double>(), d_nfb, d_bad);
  std::vector<unsigned long long> nfb((size_t)R);
  int32_t bad = 0;
  VRT_HIP(hipMemcpyAsync(nfb.data(), d_nfb, sizeof(unsigned long long) * (size_t)R, hipMemcpyDeviceToHost, s));
  VRT_HIP(hipMemcpyAsync(&bad, d_bad, 4, hipMemcpyDeviceToHost, s));
  VRT_HIP(hipStreamSynchronize(s));
  if (bad != big)
    fail(VRT_E_GRID, "site %d is not a boundary site of some ray but has no neighbour upwind in height", bad);
  g->n_fallback = 0;
  for (auto v : nfb) g->n_fallback += (int64_t)v;

  // rays that share one level schedule: the same hemisphere and the same
  // horizontal direction (rays of one azimuth at different inclinations)
  DevBuf d_peer;
  int32_t P = 0;
  if (g->shared_levels) {
    std::vector<std::vector<int32_t>> groups;
    std::vector<int32_t> gid((size_t)R, -1);
    auto hdir = [&](int32_t r, double &hx, double &hy) {
      const double x = g->h_dirs[3 * (size_t)r], y = g->h_dirs[3 * (size_t)r + 1];
      const double h = std::sqrt(x * x + y * y);
      hx = h > 1e-12 ? x / h : 0.0;
      hy = h > 1e-12 ? y / h : 0.0;
    };
    for (int32_t r = 0; r < R; ++r) {
      double hx, hy;
      hdir(r, hx, hy);
      const bool up = g->h_dirs[3 * (size_t)r + 2] > 0.0;
      for (size_t q = 0; q < groups.size() && gid[(size_t)r] < 0; ++q) {
        const int32_t o = groups[q][0];
        double ox, oy;
        hdir(o, ox, oy);
        if ((g->h_dirs[3 * (size_t)o + 2] > 0.0) == up && (hx != 0.0 || hy != 0.0) && std::fabs(hx - ox) < 1e-9 &&
            std::fabs(hy - oy) < 1e-9)
          gid[(size_t)r] = (int32_t)q;
      }
      if (gid[(size_t)r] < 0) {
        gid[(size_t)r] = (int32_t)groups.size();
        groups.push_back({});
      }
      groups[(size_t)gid[(size_t)r]].push_back(r);
    }
    for (const auto &gr : groups) P = std::max<int32_t>(P, (int32_t)gr.size());
    std::vector<int32_t> peer((size_t)R * P, -1);
    for (int32_t r = 0; r < R; ++r) {
      const auto &gr = groups[(size_t)gid[(size_t)r]];
      for (size_t q = 0; q < gr.size(); ++q) peer[(size_t)r * P + q] = gr[q];
    }
    upload(d_peer, peer.data(), peer.size(), s);
  }

  // levels by monotone relaxation, 16 passes between checks
  int32_t *level = g->d_level.as<int32_t>();
  vrt::launch_level_fill(s, RN, level);
  int64_t passes = 0;
  for (;;) {
    VRT_HIP(hipMemsetAsync(d_flags, 0, 4 * 16, s));
    for (int b = 0; b < 16; ++b)
      vrt::launch_level_relax(s, n, R, g->d_k1.as<int32_t>(), g->d_k2.as<int32_t>(), level, d_flags + b,
                              P ? d_peer.as<int32_t>() : nullptr, P);
    int32_t flags[16];
    VRT_HIP(hipMemcpyAsync(flags, d_flags, sizeof flags, hipMemcpyDeviceToHost, s));
    VRT_HIP(hipStreamSynchronize(s));
    passes += 16;
    if (flags[15] == 0) break;
    if (passes > n + 32) fail(VRT_E_DAG, "level relaxation did not converge: the upwind graph has a cycle");
  }
  int32_t lmax = 0;
  VRT_HIP(hipMemsetAsync(d_flags, 0, 4, s));
  vrt::launch_level_max(s, RN, level, d_flags);
  VRT_HIP(hipMemcpyAsync(&lmax, d_flags, 4, hipMemcpyDeviceToHost, s));
  VRT_HIP(hipStreamSynchronize(s));
  const int32_t Lmax = lmax + 1;

  // stable counting sort by (level, site index)
  const int64_t tile = 256;
  const int64_t ntiles = (n + tile - 1) / tile;
  DevBuf d_cnt, d_tot, d_lp, d_nl;
  d_cnt.alloc((size_t)R * Lmax * ntiles * 4);
  d_tot.alloc((size_t)R * Lmax * 8);
  d_lp.alloc((size_t)R * (Lmax + 1) * 4);
  d_nl.alloc((size_t)R * 4);
  VRT_HIP(hipMemsetAsync(d_cnt.p, 0, (size_t)R * Lmax * ntiles * 4, s));
  vrt::launch_level_count(s, n, R, Lmax, tile, level, d_cnt.as<int32_t>(), nullptr);
  vrt::launch_level_scan(s, R, Lmax, ntiles, d_cnt.as<int32_t>(), d_tot.as<int64_t>());
  vrt::launch_level_ptr(s, R, Lmax, d_tot.as<int64_t>(), d_lp.as<int32_t>(), d_nl.as<int32_t>());
  vrt::launch_level_scatter(s, n, R, Lmax, tile, level, d_lp.as<int32_t>(), d_cnt.as<int32_t>(),
                            g->d_order.as<int32_t>(), nullptr);
  // sweep records: the same levels, each level visited along a space-filling
  // curve of the horizontal position, so neighbouring records share upwind sites
  DevBuf d_rec_order, d_visit;
  const int32_t *rec_order = g->d_order.as<int32_t>();
  if (g->record_order == 1 && n > 1) {
    std::vector<uint64_t> key = morton_codes(g);
    for (int64_t i = 0; i < n; ++i) key[(size_t)i] = (key[(size_t)i] << 31) | (uint64_t)i;
    std::sort(key.begin(), key.end());
    std::vector<int32_t> visit((size_t)n);
    for (int64_t i = 0; i < n; ++i) visit[(size_t)i] = (int32_t)(key[(size_t)i] & 0x7fffffffu);
    upload(d_visit, visit.data(), visit.size(), s);
    d_rec_order.alloc((size_t)RN * 4);
    VRT_HIP(hipMemsetAsync(d_cnt.p, 0, (size_t)R * Lmax * ntiles * 4, s));
    vrt::launch_level_count(s, n, R, Lmax, tile, level, d_cnt.as<int32_t>(), d_visit.as<int32_t>());
    vrt::launch_level_scan(s, R, Lmax, ntiles, d_cnt.as<int32_t>(), d_tot.as<int64_t>());
    vrt::launch_level_scatter(s, n, R, Lmax, tile, level, d_lp.as<int32_t>(), d_cnt.as<int32_t>(),
                              d_rec_order.as<int32_t>(), d_visit.as<int32_t>());
    rec_order = d_rec_order.as<int32_t>();
    VRT_HIP(hipStreamSynchronize(s));  // visit lives in host memory until the copy is done
  }
  std::vector<int32_t> lp((size_t)R * (Lmax + 1));
  g->n_levels.assign((size_t)R, 0);
  VRT_HIP(hipMemcpyAsync(lp.data(), d_lp.p, lp.size() * 4, hipMemcpyDeviceToHost, s));
  VRT_HIP(hipMemcpyAsync(g->n_levels.data(), d_nl.p, (size_t)R * 4, hipMemcpyDeviceToHost, s));
  VRT_HIP(hipStreamSynchronize(s));
  g->level_ptr.assign((size_t)R, {});
  for (int32_t r = 0; r < R; ++r) {
    const int32_t L = g->n_levels[(size_t)r];
    g->level_ptr[(size_t)r].assign(lp.begin() + (int64_t)r * (Lmax + 1), lp.begin() + (int64_t)r * (Lmax + 1) + L + 1);
    if (g->level_ptr[(size_t)r].back() != n) fail(VRT_E_DAG, "schedule of ray %d does not cover every site", r);
  }

  // step-major record layout: step s holds level s of ray 0, 1, ..., R-1
  g->n_steps = n > 0 ? *std::max_element(g->n_levels.begin(), g->n_levels.end()) : 0;
  const int32_t NS = g->n_steps;
  g->seg_off.assign((size_t)NS * R, 0);
  g->seg_cnt.assign((size_t)NS * R, 0);
  g->step_ptr.assign((size_t)NS + 1, 0);
  int64_t acc = 0;
  for (int32_t st = 0; st < NS; ++st) {
    g->step_ptr[(size_t)st] = acc;
    for (int32_t r = 0; r < R; ++r) {
      const auto &p = g->level_ptr[(size_t)r];
      const int64_t c = st < g->n_levels[(size_t)r] ? (int64_t)p[(size_t)st + 1] - p[(size_t)st] : 0;
      g->seg_off[(size_t)st * R + r] = acc;
      g->seg_cnt[(size_t)st * R + r] = c;
      acc += c;
    }
  }
  g->step_ptr[(size_t)NS] = acc;
  g->n_rec = acc;
  build_affinity(g);
  DevBuf d_seg;
  upload(d_seg, g->seg_off.data(), g->seg_off.size(), s);
  g->d_ri.alloc((size_t)RN * sizeof(int4));
  g->d_rf32.alloc((size_t)RN * sizeof(vrt::RecF32));
  g->d_rf64.alloc((size_t)RN * sizeof(vrt::RecF64));
  vrt::launch_pack(s, n, R, Lmax, rec_order, level, d_lp.as<int32_t>(), d_seg.as<int64_t>(),
                   g->d_k1.as<int32_t>(), g->d_k2.as<int32_t>(), g->d_w1.as<double>(), g->d_ds1.as<double>(),
                   g->d_ds2.as<double>(), g->d_dirs.as<double>(), g->d_ri.as<int4>(), g->d_rf32.as<vrt::RecF32>(),
                   g->d_rf64.as<vrt::RecF64>());
  VRT_HIP(hipStreamSynchronize(s));
  g->interleaved_built = 0;
  if (g->interleave) build_interleaved(g);
  g->down_built = false;
  if (g->segment) build_downwind(g);
  g->ck_levels = 0;  // the checkpoint table names record indices
}

template <typename T> T *intensity_buffer(vrt_grid g, int32_t nl, void *I_rays) {
  if (I_rays) return static_cast<T *>(I_rays);
  const size_t bytes = (size_t)g->R * (size_t)g->n * (size_t)nl * sizeof(T);
  if (bytes > g->d_Iscr.bytes) {
    g->drop_graphs();  // captured launches may point into the old scratch
    g->d_Iscr.alloc(bytes);
  }
  return g->d_Iscr.as<T>();
}

// Rows of the sign-encoded persistent sweep: a block of their own (no other
// mode writes it), refilled with zeros of the current epoch's sign whenever its
// layout changes or an error was acknowledged, so that no element left from
// another layout or an abandoned sweep reads as written by the next epoch.
void ensure_flags(vrt_grid g);
template <typename T> T *sign_buffer(vrt_grid g, int32_t nl) {
  ensure_flags(g);
  const int64_t count = (int64_t)g->R * g->n * nl;
  const int64_t key[4] = {(int64_t)sizeof(T), nl, g->R, g->n};
  bool fill = false;
  if ((size_t)count * sizeof(T) > g->d_Isgn.bytes) {
    g->d_Isgn.alloc((size_t)count * sizeof(T));
    fill = true;
  }
  for (int k = 0; k < 4; ++k) fill = fill || g->sgn_key[k] != key[k];
  if (fill) {
    vrt::launch_sign_fill<T>(g->ctx->stream, g->d_Isgn.as<T>(), count, g->d_epoch.as<int32_t>());
    for (int k = 0; k < 4; ++k) g->sgn_key[k] = key[k];
  }
  return g->d_Isgn.as<T>();
}

// Runs one launch, bracketed by timing events when the context profiles
// (never inside a graph capture: `timed` is false there).
template <typename F> void timed_launch(vrt_ctx ctx, hipStream_t s, bool timed, int kernel, int64_t units, F &&launch) {
  if (!timed) {
    launch();
    return;
  }
  vrt_ctx_s::Timed t{kernel, nullptr, nullptr, units};
  VRT_HIP(hipEventCreate(&t.start));
  VRT_HIP(hipEventCreate(&t.stop));
  VRT_HIP(hipEventRecord(t.start, s));
  launch();
  VRT_HIP(hipEventRecord(t.stop, s));
  ctx->pending.push_back(t);
}

// per-(ray, site) epoch stamps, each ray's block padded to whole 128-byte
// cache lines, and the epoch / device-error / registration words
int64_t flag_ld(vrt_grid g) { return (g->n + 31) / 32 * 32; }

void ensure_flags(vrt_grid g) {
  if (g->d_flags.p) return;
  const size_t bytes = (size_t)g->R * (size_t)flag_ld(g) * 4;
  g->d_flags.alloc(bytes);
  VRT_HIP(hipMemsetAsync(g->d_flags.p, 0, bytes, g->ctx->stream));
  g->d_epoch.alloc(64);
  VRT_HIP(hipMemsetAsync(g->d_epoch.p, 0, 64, g->ctx->stream));
}

// Reads and acknowledges the persistent sweeps' device error word (callers
// synchronise the stream first). A set word clears the word and the layout
// key of the sign-encoded rows, so those rows are refilled with zeros of the
// current epoch's sign before their next use: a sweep that stopped early or did
// not run left rows of an older sign, which a later epoch of the same sign
// would otherwise read as written. Value 2 (a negative or NaN intensity that
// the sign encoding cannot carry) is reported as VRT_E_NUMERIC, value 1 (a
// bounded wait gave up) as VRT_E_TIMEOUT; `iter` > 0 names the iteration.
void take_device_error(vrt_grid g, int32_t iter) {
  if (!g->d_epoch.p) return;
  int32_t err = 0;
  VRT_HIP(hipMemcpy(&err, g->d_epoch.as<int32_t>() + 1, 4, hipMemcpyDeviceToHost));
  if (err == 0) return;
  VRT_HIP(hipMemset(g->d_epoch.as<int32_t>() + 1, 0, 4));
  for (int k = 0; k < 4; ++k) g->sgn_key[k] = 0;
  ++g->solution_id;  // the last solution's rows may be of no single epoch
  char at[48] = "";
  if (iter > 0) snprintf(at, sizeof at, " at iteration %d", iter);
  if (err & 2)
    fail(VRT_E_NUMERIC, "negative or NaN intensity in the sign-encoded persistent sweep%s (it needs I >= 0; pass "
                        "I_rays or use another execution mode for such inputs)", at);
  fail(VRT_E_TIMEOUT, "a bounded wait of the persistent sweep gave up%s (spin cap %lld)", at, (long long)g->spin_cap);
}

// Wave items of the persistent sweep: the (level step, ray) segments in step
// order, cut into at most spw records, cnt = record count + 256 x ray; or, with
// `mixed`, each level step of the interleaved record copy cut into spw
// records whatever their rays (cnt = record count).
const vrt::PersistItems &persistent_items(vrt_grid g, int32_t spw, bool mixed = false) {
  const int key = spw + (mixed ? 1024 : 0);
  auto it = g->persist_items.find(key);
  if (it != g->persist_items.end()) return *it->second;
  const int32_t R = g->R;
  if (R >= (1 << 23)) fail(VRT_E_ARG, "persistent sweep: too many rays");
  std::vector<int64_t> rec;
  std::vector<int32_t> cnt;
  for (int32_t st = 0; st < g->n_steps; ++st) {
    if (mixed) {
      const int64_t b = g->step_ptr[(size_t)st], e = g->step_ptr[(size_t)st + 1];
      for (int64_t r = b; r < e; r += spw) {
        rec.push_back(r);
        cnt.push_back((int32_t)std::min<int64_t>(spw, e - r));
      }
      continue;
    }
    for (int32_t ray = 0; ray < R; ++ray) {
      const int64_t b = g->seg_off[(size_t)st * R + ray], e = b + g->seg_cnt[(size_t)st * R + ray];
      for (int64_t r = b; r < e; r += spw) {
        rec.push_back(r);
        cnt.push_back((int32_t)std::min<int64_t>(spw, e - r) + 256 * ray);
      }
    }
  }
  std::unique_ptr<vrt::PersistItems> p(new vrt::PersistItems);
  p->spw = spw;
  p->n_items = (int64_t)rec.size();
  upload(p->rec, rec.data(), rec.size(), g->ctx->stream);
  upload(p->cnt, cnt.data(), cnt.size(), g->ctx->stream);
  ensure_flags(g);
  VRT_HIP(hipStreamSynchronize(g->ctx->stream));  // host tables are local
  auto &ref = *p;
  g->persist_items.emplace(key, std::move(p));
  return ref;
}

// The sweeps of every ray (no angle quadrature). The input rows of site i
// (chi, S, Ib, It) start at i cs (cs = 0: nl, arrays of n x nl).
template <typename T>
void enqueue_sweep(vrt_grid g, hipStream_t s, vrt_exec ex, int32_t nl, const T *chi, const T *S, const T *Ib,
                   const T *It, T *I, bool sign = false, int64_t cs = 0) {
  const int32_t R = g->R;
  const int64_t n = g->n;
  if (cs == 0) cs = nl;
  // the plane kernels of the regular grid read rows of nl entries
  if (g->kind != 0 && cs != nl) fail(VRT_E_ARG, "a regular grid takes chi and S rows of n_lambda entries");
  vrt_ctx ctx = g->ctx;
  const bool tm = ctx->profiling && ex != VRT_EXEC_GRAPH && s == ctx->stream;
  if (g->kind == 0 && g->segment == 1) {
    const int4 *ri = g->d_ri.as<int4>();
    const auto *rf = records<T>(g);
    auto sweep = [&](const int4 *rix, decltype(rf) rfx, int64_t b, int64_t c) {
      if (c <= 0) return;
      timed_launch(ctx, s, tm, 0, c * nl, [&] {
        vrt::launch_bezier_sweep<T>(s, rix, rfx, b, c, nl, cs, n, g->d_q1.as<int32_t>(), g->d_q2.as<int32_t>(),
                                    g->d_qw1.as<double>(), g->d_qd1.as<double>(), g->d_qd2.as<double>(), chi, S, Ib,
                                    It, I, g->xcd_chunks);
      });
    };
    if (ex == VRT_EXEC_PERSISTENT) {
      const vrt::PersistItems &items = persistent_items(g, vrt::bezier_records_per_wave());
      int32_t *words = g->d_epoch.as<int32_t>();
      vrt::launch_persist_begin(s, words);
      timed_launch(ctx, s, tm, 0, g->n_rec * nl, [&] {
        vrt::launch_persistent_bezier<T>(s, items, g->persist_max_blocks, ri, rf, nl, cs, n, g->d_q1.as<int32_t>(),
                                         g->d_q2.as<int32_t>(), g->d_qw1.as<double>(), g->d_qd1.as<double>(),
                                         g->d_qd2.as<double>(), chi, S, Ib, It, I, flag_ld(g),
                                         g->d_flags.as<int32_t>(), words, g->spin_cap);
      });
    } else if (ex == VRT_EXEC_PLAIN) {
      for (int32_t r = 0; r < R; ++r)
        for (int32_t st = 0; st < g->n_levels[(size_t)r]; ++st)
          sweep(ri, rf, g->seg_off[(size_t)st * R + r], g->seg_cnt[(size_t)st * R + r]);
    } else {
      // step-wide launches read the interleaved copy when there is one
      const int4 *rix = ri;
      auto rfx = rf;
      if (g->interleave && g->interleaved_built == g->interleave) {
        rix = g->d_ri_x.as<int4>();
        rfx = sizeof(T) == 4 ? reinterpret_cast<decltype(rf)>(g->d_rf32_x.p)
                             : reinterpret_cast<decltype(rf)>(g->d_rf64_x.p);
      }
      for (int32_t st = 0; st < g->n_steps; ++st)
        sweep(rix, rfx, g->step_ptr[(size_t)st], g->step_ptr[(size_t)st + 1] - g->step_ptr[(size_t)st]);
    }
  } else if (g->kind == 0 && ex == VRT_EXEC_PERSISTENT) {
    const bool aligned = vrt::al16(chi) && vrt::al16(S) && vrt::al16(Ib) && vrt::al16(It) && vrt::al16(I);
    // the interleaved record copy, when there is one: wave items then take
    // records of several rays
    const bool mixed = g->interleave && g->interleaved_built == g->interleave;
    const vrt::PersistItems &items =
        persistent_items(g, vrt::persistent_records_per_wave(nl, sizeof(T), aligned, cs), mixed);
    const int4 *rix = mixed ? g->d_ri_x.as<int4>() : g->d_ri.as<int4>();
    const auto *rfx = records<T>(g);
    if (mixed)
      rfx = sizeof(T) == 4 ? reinterpret_cast<decltype(rfx)>(g->d_rf32_x.p) : reinterpret_cast<decltype(rfx)>(g->d_rf64_x.p);
    int32_t *words = g->d_epoch.as<int32_t>();
    vrt::launch_persist_begin(s, words, sign);
    timed_launch(ctx, s, tm, 0, g->n_rec * nl, [&] {
      vrt::launch_persistent_sweep<T>(s, items, g->persist_max_blocks, rix, rfx, nl, cs, n, flag_ld(g), chi, S, Ib,
                                      It, I, g->d_flags.as<int32_t>(), words, g->spin_cap, sign, mixed ? R : 0);
    });
  } else if (g->kind == 0) {
    const int4 *ri = g->d_ri.as<int4>();
    const auto *rf = records<T>(g);
    const int32_t xc = g->xcd_chunks;
    // level step st of the step-major records; the pipelined kernel takes the
    // interior steps (st >= 1) of the step-wide modes
    auto sweep = [&](int32_t st, int64_t b, int64_t c) {
      if (c <= 0) return;
      const int32_t pp = (ex == VRT_EXEC_PLAIN || st == 0) ? 0 : g->pipe;
      timed_launch(ctx, s, tm, 0, c * nl, [&] {
        vrt::launch_sweep<T>(s, ri, rf, b, c, nl, cs, n, chi, S, Ib, It, I, xc, 0, nullptr, 0, g->lane_bytes, pp);
      });
    };
    if (ex == VRT_EXEC_PLAIN) {
      for (int32_t r = 0; r < R; ++r)
        for (int32_t st = 0; st < g->n_levels[(size_t)r]; ++st)
          sweep(st, g->seg_off[(size_t)st * R + r], g->seg_cnt[(size_t)st * R + r]);
    } else if (g->ray_affinity) {
      const int64_t *xt = g->d_xtab.as<int64_t>();
      const size_t per = (size_t)vrt::kDies * g->xk * 2;
      for (int32_t st = 0; st < g->n_steps; ++st) {
        const int64_t c = g->xmax[(size_t)st];
        if (c <= 0) continue;
        const int64_t units = (g->step_ptr[(size_t)st + 1] - g->step_ptr[(size_t)st]) * nl;
        timed_launch(ctx, s, tm, 0, units, [&] {
          vrt::launch_sweep<T>(s, ri, rf, 0, c, nl, cs, n, chi, S, Ib, It, I, 0, 0, xt + per * st, g->xk,
                               g->lane_bytes);
        });
      }
    } else if (g->chains > 1 && R > 1) {
      // rays never read each other's intensities: split them into K contiguous
      // ranges, each swept level by level on a stream of its own, so one
      // chain's launch latency overlaps the other chains' work
      const int32_t K = std::min<int32_t>(g->chains, R);
      ctx->ensure_aux(K - 1);
      VRT_HIP(hipEventRecord(ctx->fork_ev, s));
      for (int32_t c = 1; c < K; ++c) VRT_HIP(hipStreamWaitEvent(ctx->aux[(size_t)c - 1], ctx->fork_ev, 0));
      for (int32_t st = 0; st < g->n_steps; ++st) {
        for (int32_t c = 0; c < K; ++c) {
          const int32_t r0 = (int32_t)((int64_t)c * R / K), r1 = (int32_t)((int64_t)(c + 1) * R / K);
          const int64_t b = g->seg_off[(size_t)st * R + r0];
          const int64_t e = g->seg_off[(size_t)st * R + r1 - 1] + g->seg_cnt[(size_t)st * R + r1 - 1];
          if (e <= b) continue;
          hipStream_t sc = c == 0 ? s : ctx->aux[(size_t)c - 1];
          timed_launch(ctx, sc, tm, 0, (e - b) * nl,
                       [&] {
                         vrt::launch_sweep<T>(sc, ri, rf, b, e - b, nl, cs, n, chi, S, Ib, It, I, xc, 0, nullptr, 0,
                                              g->lane_bytes, st > 0 ? g->pipe : 0);
                       });
        }
      }
      for (int32_t c = 1; c < K; ++c) {
        VRT_HIP(hipEventRecord(ctx->join_ev[(size_t)c - 1], ctx->aux[(size_t)c - 1]));
        VRT_HIP(hipStreamWaitEvent(s, ctx->join_ev[(size_t)c - 1], 0));
      }
    } else if (g->ray_groups > 1 && R > 1) {
      // contiguous ray ranges swept one after another: each level step then
      // touches fewer rows, so an upwind row is more likely still cached
      const int32_t K = std::min<int32_t>(g->ray_groups, R);
      for (int32_t c = 0; c < K; ++c) {
        const int32_t r0 = (int32_t)((int64_t)c * R / K), r1 = (int32_t)((int64_t)(c + 1) * R / K);
        for (int32_t st = 0; st < g->n_steps; ++st) {
          const int64_t b = g->seg_off[(size_t)st * R + r0];
          const int64_t e = g->seg_off[(size_t)st * R + r1 - 1] + g->seg_cnt[(size_t)st * R + r1 - 1];
          sweep(st, b, e - b);
        }
      }
    } else {
      const int4 *rix = ri;
      const auto *rfx = rf;
      if (g->interleave && g->interleaved_built == g->interleave) {
        rix = g->d_ri_x.as<int4>();
        rfx = sizeof(T) == 4 ? reinterpret_cast<decltype(rf)>(g->d_rf32_x.p) : reinterpret_cast<decltype(rf)>(g->d_rf64_x.p);
      }
      for (int32_t st = 0; st < g->n_steps; ++st) {
        const int64_t b = g->step_ptr[(size_t)st], c = g->step_ptr[(size_t)st + 1] - b;
        if (c <= 0) continue;
        timed_launch(ctx, s, tm, 0, c * nl, [&] {
          vrt::launch_sweep<T>(s, rix, rfx, b, c, nl, cs, n, chi, S, Ib, It, I, xc, 0, nullptr, 0, g->lane_bytes,
                               st > 0 ? g->pipe : 0);
        });
      }
    }
  } else {
    const double *z = g->d_z.as<double>(), *dirs = g->d_dirs.as<double>();
    const int64_t plane = (int64_t)g->nx * g->ny;
    auto planes = [&](int32_t st, int32_t rb, int32_t rc) {
      timed_launch(ctx, s, tm, 2, plane * rc * nl, [&] {
        vrt::launch_regular<T>(s, st, rb, rc, g->nx, g->ny, g->nz, g->dx, g->dy, z, dirs, nl, chi, S, Ib, It, I,
                               g->regular_tiled == 1 || (g->regular_tiled == 2 && sizeof(T) == 8), g->xcd_chunks);
      });
    };
    if (ex == VRT_EXEC_PLAIN) {
      for (int32_t r = 0; r < R; ++r)
        for (int32_t st = 0; st < g->nz; ++st) planes(st, r, 1);
    } else {
      for (int32_t st = 0; st < g->nz; ++st) planes(st, 0, R);
    }
  }
}

template <typename T>
void enqueue_fs(vrt_grid g, hipStream_t s, vrt_exec ex, int32_t nl, const T *chi, const T *S, const T *Ib,
                const T *It, T *J, T *I, bool sign = false, int64_t cs = 0) {
  enqueue_sweep<T>(g, s, ex, nl, chi, S, Ib, It, I, sign, cs);
  vrt_ctx ctx = g->ctx;
  const bool tm = ctx->profiling && ex != VRT_EXEC_GRAPH && s == ctx->stream;
  const int32_t R = g->R;
  const int64_t n = g->n;
  timed_launch(ctx, s, tm, 1, (int64_t)R * n * nl,
               [&] {
                 vrt::launch_jreduce<T>(s, I, R, n * nl, g->d_w.as<double>(), J, sign,
                                        sign ? g->d_epoch.as<int32_t>() + 1 : nullptr);
               });
}

// Per-ray dependents lists: for every site k, the sites d whose forward update
// read k, in increasing d (then line) order, with the weight and length of
// that line. Built on the host from the selection, once per quadrature.
void build_dependents(vrt_grid g) {
  if (g->deps_built) return;
  const int64_t n = g->n;
  const int32_t R = g->R;
  const size_t RN = (size_t)R * (size_t)n;
  hipStream_t s = g->ctx->stream;
  std::vector<int32_t> k1(RN), k2(RN);
  std::vector<double> w1(RN), d1(RN), d2(RN);
  VRT_HIP(hipMemcpyAsync(k1.data(), g->d_k1.p, RN * 4, hipMemcpyDeviceToHost, s));
  VRT_HIP(hipMemcpyAsync(k2.data(), g->d_k2.p, RN * 4, hipMemcpyDeviceToHost, s));
  VRT_HIP(hipMemcpyAsync(w1.data(), g->d_w1.p, RN * 8, hipMemcpyDeviceToHost, s));
  VRT_HIP(hipMemcpyAsync(d1.data(), g->d_ds1.p, RN * 8, hipMemcpyDeviceToHost, s));
  VRT_HIP(hipMemcpyAsync(d2.data(), g->d_ds2.p, RN * 8, hipMemcpyDeviceToHost, s));
  VRT_HIP(hipStreamSynchronize(s));
  std::vector<int64_t> ptr((size_t)R * (size_t)(n + 1), 0);
  int64_t total = 0;
  for (int32_t r = 0; r < R; ++r) {
    int64_t *p = ptr.data() + (size_t)r * (size_t)(n + 1);
    const size_t o = (size_t)r * (size_t)n;
    for (int64_t d = 0; d < n; ++d) {
      if (k1[o + d] >= 0) p[k1[o + d] + 1]++;
      if (k2[o + d] >= 0) p[k2[o + d] + 1]++;
    }
    p[0] = total;
    for (int64_t k = 0; k < n; ++k) p[k + 1] += p[k];
    total = p[n];
  }
  std::vector<int32_t> site((size_t)total);
  std::vector<vrt::RecF32> r32((size_t)total);
  std::vector<vrt::RecF64> r64((size_t)total);
  std::vector<int64_t> cur(ptr);
  for (int32_t r = 0; r < R; ++r) {
    int64_t *c = cur.data() + (size_t)r * (size_t)(n + 1);
    const size_t o = (size_t)r * (size_t)n;
    for (int64_t d = 0; d < n; ++d) {
      const bool two = k2[o + d] >= 0;
      for (int j = 0; j < 2; ++j) {
        const int32_t k = j == 0 ? k1[o + d] : k2[o + d];
        if (k < 0) continue;
        const double w = two ? (j == 0 ? w1[o + d] : 1.0 - w1[o + d]) : 1.0;
        const double ds = j == 0 ? d1[o + d] : d2[o + d];
        const int64_t t = c[k]++;
        site[(size_t)t] = (int32_t)d;
        r32[(size_t)t] = vrt::RecF32{(float)w, (float)ds, 0.0f, 0.0f};
        r64[(size_t)t] = vrt::RecF64{w, ds, 0.0, 0.0};
      }
    }
  }
  upload(g->d_dep_ptr, ptr.data(), ptr.size(), s);
  upload(g->d_dep_site, site.data(), site.size(), s);
  upload(g->d_dep_rf32, r32.data(), r32.size(), s);
  upload(g->d_dep_rf64, r64.data(), r64.size(), s);
  VRT_HIP(hipStreamSynchronize(s));
  g->deps_built = true;
}

// Checkpoint plan of the reverse sweep for level chunks of K steps (chunk c =
// steps [cK, cK + K)) and ray groups of `group` rays. Within a group, the
// records of one chunk get consecutive chunk slots (the chunk buffer holds one
// chunk's rows at a time), and every (ray, site) whose row is read by a record
// of a later chunk gets a frontier slot (its row is kept for the rest of the
// reverse sweep). A record's upwind row lies in the chunk buffer when the
// upwind site is in the same chunk, else in the frontier buffer (upwind sites
// sit at lower level steps, so never in a later chunk). Host work O(R n).
void build_checkpoints(vrt_grid g, int32_t K, int32_t group) {
  if (g->ck_levels == K && g->ck_group == group) return;
  const int64_t n = g->n;
  const int32_t R = g->R, NS = g->n_steps;
  hipStream_t s = g->ctx->stream;
  std::vector<int4> ri((size_t)g->n_rec);
  VRT_HIP(hipMemcpyAsync(ri.data(), g->d_ri.p, ri.size() * sizeof(int4), hipMemcpyDeviceToHost, s));
  VRT_HIP(hipStreamSynchronize(s));
  std::vector<int4> tab((size_t)g->n_rec, make_int4(0, -1, 0, 0));
  std::vector<int64_t> rec_of;
  std::vector<int32_t> chunk_of, fslot;
  int64_t max_rows = 0, max_front = 0;
  for (int32_t r0 = 0; r0 < R; r0 += group) {
    const int32_t gc = std::min(group, R - r0);
    const size_t GN = (size_t)gc * (size_t)n;
    rec_of.assign(GN, -1);
    chunk_of.assign(GN, 0);
    fslot.assign(GN, -1);
    // chunk slots, and the record and chunk of every (ray, site) of the group
    for (int32_t c0 = 0; c0 < NS; c0 += K) {
      int64_t slot = 0;
      for (int32_t st = c0; st < std::min(c0 + K, NS); ++st)
        for (int32_t r = r0; r < r0 + gc; ++r) {
          const int64_t b = g->seg_off[(size_t)st * R + r], c = g->seg_cnt[(size_t)st * R + r];
          for (int64_t rec = b; rec < b + c; ++rec) {
            const size_t key = (size_t)(r - r0) * (size_t)n + (size_t)ri[(size_t)rec].x;
            rec_of[key] = rec;
            chunk_of[key] = c0 / K;
            tab[(size_t)rec].x = (int32_t)slot++;
          }
        }
      max_rows = std::max(max_rows, slot);
    }
    for (size_t key = 0; key < GN; ++key)
      if (rec_of[key] < 0) fail(VRT_E_STATE, "the schedule misses a site of ray %d", r0 + (int32_t)(key / (size_t)n));
    // frontier rows: read from a later chunk
    for (size_t key = 0; key < GN; ++key) {
      const int4 q = ri[(size_t)rec_of[key]];
      const size_t base = key - key % (size_t)n;
      for (int32_t u : {q.y, q.z})
        if (u >= 0 && chunk_of[base + (size_t)u] < chunk_of[key]) fslot[base + (size_t)u] = 0;
    }
    int64_t front = 0;
    for (size_t key = 0; key < GN; ++key)
      if (fslot[key] == 0) fslot[key] = (int32_t)(front++) + 1;  // stored + 1 until the table is written
    max_front = std::max(max_front, front);
    for (size_t key = 0; key < GN; ++key) {
      const int64_t rec = rec_of[key];
      const int4 q = ri[(size_t)rec];
      const size_t base = key - key % (size_t)n;
      int4 &t = tab[(size_t)rec];
      t.y = fslot[key] > 0 ? fslot[key] - 1 : -1;
      auto loc = [&](int32_t u) -> int32_t {
        if (u < 0) return 0;
        const size_t ku = base + (size_t)u;
        if (chunk_of[ku] == chunk_of[key]) return tab[(size_t)rec_of[ku]].x;
        return -fslot[ku];  // -(frontier slot + 1)
      };
      t.z = loc(q.y);
      t.w = q.z >= 0 ? loc(q.z) : t.z;
    }
  }
  if (max_rows > INT32_MAX || max_front >= INT32_MAX) fail(VRT_E_ARG, "checkpoint buffers above 2^31 rows");
  upload(g->d_ck, tab.data(), tab.size(), s);
  VRT_HIP(hipStreamSynchronize(s));
  g->ck_levels = K;
  g->ck_group = group;
  g->ck_chunk_rows = max_rows;
  g->ck_front_rows = max_front;
}

// Wave items of the persistent reverse sweep of rays [r0, r0 + gc) for `spw`
// records per wave: the (level step, ray) segments in decreasing step order,
// each cut separately; cnt holds the record count + 256 x (ray - r0).
const vrt::PersistItems &reverse_items(vrt_grid g, int32_t spw, int32_t r0, int32_t gc) {
  const int64_t key = ((int64_t)spw << 40) | ((int64_t)r0 << 20) | (int64_t)gc;
  auto it = g->reverse_items.find(key);
  if (it != g->reverse_items.end()) return *it->second;
  const int32_t R = g->R;
  std::vector<int64_t> rec;
  std::vector<int32_t> cnt;
  for (int32_t st = g->n_steps - 1; st >= 0; --st) {
    for (int32_t ray = r0; ray < r0 + gc; ++ray) {
      const int64_t b = g->seg_off[(size_t)st * R + ray], e = b + g->seg_cnt[(size_t)st * R + ray];
      for (int64_t r = b; r < e; r += spw) {
        rec.push_back(r);
        cnt.push_back((int32_t)std::min<int64_t>(spw, e - r) + 256 * (ray - r0));
      }
    }
  }
  std::unique_ptr<vrt::PersistItems> p(new vrt::PersistItems);
  p->spw = spw;
  p->n_items = (int64_t)rec.size();
  upload(p->rec, rec.data(), rec.size(), g->ctx->stream);
  upload(p->cnt, cnt.data(), cnt.size(), g->ctx->stream);
  ensure_flags(g);
  VRT_HIP(hipStreamSynchronize(g->ctx->stream));  // host tables are local
  auto &ref = *p;
  g->reverse_items.emplace(key, std::move(p));
  return ref;
}

template <typename T> const typename vrt::RecOf<T>::type *dep_records(vrt_grid g);
template <> const vrt::RecF32 *dep_records<float>(vrt_grid g) { return g->d_dep_rf32.as<vrt::RecF32>(); }
template <> const vrt::RecF64 *dep_records<double>(vrt_grid g) { return g->d_dep_rf64.as<vrt::RecF64>(); }

// Reverse sweep over ray groups of `group` rays: the forward intensities come
// from I_rays when given, else each group's are recomputed first; the group's
// adjoint contributions are summed into double accumulators.
template <typename T>
void formal_solution_vjp(vrt_grid g, int32_t nl, const T *chi, const T *S, const T *Ib, const T *It,
                         const T *I_rays, const T *gI, const T *gJ, T *o_chi, T *o_S, T *o_Ib, T *o_It,
                         int32_t group, int32_t ckpt) {
  build_dependents(g);
  hipStream_t s = g->ctx->stream;
  const int64_t n = g->n;
  const int32_t R = g->R;
  const int64_t nn = n * nl;
  if (group <= 0 || group > R) group = R;
  const size_t gbytes = (size_t)group * (size_t)nn * sizeof(T);
  // level-chunk checkpoints replace the group's full forward rows
  const bool ck = !I_rays && ckpt > 0;
  T *Ich = nullptr, *Ifr = nullptr;
  if (ck) {
    build_checkpoints(g, std::min(ckpt, std::max(g->n_steps, 1)), group);
    g->d_vI.release();
    g->d_vIch.alloc((size_t)std::max<int64_t>(g->ck_chunk_rows, 1) * (size_t)nl * sizeof(T));
    g->d_vIfr.alloc((size_t)std::max<int64_t>(g->ck_front_rows, 1) * (size_t)nl * sizeof(T));
    Ich = g->d_vIch.as<T>();
    Ifr = g->d_vIfr.as<T>();
  } else if (!I_rays) {
    g->d_vI.alloc(gbytes);
  }
  g->d_vIbar.alloc(gbytes);
  g->d_vSbar.alloc(gbytes);
  g->d_vCbar.alloc(gbytes);
  g->d_vacc.alloc((size_t)nn * 4 * sizeof(double));
  double *acc = g->d_vacc.as<double>();
  vrt::launch_fill_zero<double>(s, nn * 4, acc);
  T *Ibar = g->d_vIbar.as<T>(), *Sbar = g->d_vSbar.as<T>(), *Cbar = g->d_vCbar.as<T>();
  const int4 *ri = g->d_ri.as<int4>();
  const auto *rf = records<T>(g);
  // (the interleaved record copy was measured slower here: the reverse sweep
  // gathers its dependents' adjoint rows ray by ray)
  for (int32_t r0 = 0; r0 < R; r0 += group) {
    const int32_t gc = std::min(group, R - r0);
    auto seg = [&](int32_t st, int64_t &b, int64_t &c) {
      b = g->seg_off[(size_t)st * R + r0];
      const int32_t rl = r0 + gc - 1;
      c = g->seg_off[(size_t)st * R + rl] + g->seg_cnt[(size_t)st * R + rl] - b;
    };
    if (ck) {
      // forward over every step, keeping the frontier rows (and the last
      // chunk's rows in the chunk buffer); then chunk by chunk downwards:
      // recompute the chunk's rows from the frontier, then its reverse steps
      const int4 *tab = g->d_ck.as<int4>();
      const int32_t K = g->ck_levels;
      for (int32_t st = 0; st < g->n_steps; ++st) {
        int64_t b, c;
        seg(st, b, c);
        vrt::launch_sweep_ck<T>(s, ri, rf, tab, b, c, nl, chi, S, Ib, It, Ich, Ifr);
      }
      const int32_t last = g->n_steps > 0 ? (g->n_steps - 1) / K : 0;
      for (int32_t cc = last; cc >= 0; --cc) {
        const int32_t s0 = cc * K, s1 = std::min(s0 + K, g->n_steps);
        if (cc != last)
          for (int32_t st = s0; st < s1; ++st) {
            int64_t b, c;
            seg(st, b, c);
            vrt::launch_sweep_ck<T>(s, ri, rf, tab, b, c, nl, chi, S, Ib, It, Ich, Ifr);
          }
        for (int32_t st = s1 - 1; st >= s0; --st) {
          int64_t b, c;
          seg(st, b, c);
          vrt::launch_reverse<T>(s, ri, rf, b, c, nl, n, r0, g->d_dep_ptr.as<int64_t>(),
                                 g->d_dep_site.as<int32_t>(), dep_records<T>(g), chi, S, Ich, gI, gJ,
                                 g->d_w.as<double>(), Ibar, Sbar, Cbar, tab, Ich, Ifr);
        }
      }
      vrt::launch_reverse_reduce<T>(s, n, nl, r0, gc, g->d_dirs.as<double>(), g->d_wall.as<uint8_t>(), Ibar, Sbar,
                                    Cbar, acc, acc + nn, acc + 2 * nn, acc + 3 * nn);
      continue;
    }
    const T *Ifw;
    if (I_rays) {
      Ifw = I_rays + (size_t)r0 * (size_t)nn;
    } else {
      T *Iw = g->d_vI.as<T>();
      for (int32_t st = 0; st < g->n_steps; ++st) {
        int64_t b, c;
        seg(st, b, c);
        vrt::launch_sweep<T>(s, ri, rf, b, c, nl, nl, n, chi, S, Ib, It, Iw, g->xcd_chunks, r0);
      }
      Ifw = Iw;
    }
    if (g->reverse_persistent) {
      const bool aligned = vrt::al16(chi) && vrt::al16(S) && vrt::al16(Ifw) && vrt::al16(gI) && vrt::al16(gJ) &&
                           vrt::al16(Ibar) && vrt::al16(Sbar) && vrt::al16(Cbar);
      const vrt::PersistItems &items =
          reverse_items(g, vrt::reverse_records_per_wave(nl, sizeof(T), aligned), r0, gc);
      int32_t *words = g->d_epoch.as<int32_t>();
      vrt::launch_persist_begin(s, words);
      vrt::launch_persistent_reverse<T>(s, items, g->persist_max_blocks, ri, rf, nl, n, r0,
                                        g->d_dep_ptr.as<int64_t>(), g->d_dep_site.as<int32_t>(), dep_records<T>(g),
                                        chi, S, Ifw, gI, gJ, g->d_w.as<double>(), Ibar, Sbar, Cbar, flag_ld(g),
                                        g->d_flags.as<int32_t>(), words, g->spin_cap);
    } else {
      for (int32_t st = g->n_steps - 1; st >= 0; --st) {
        int64_t b, c;
        seg(st, b, c);
        vrt::launch_reverse<T>(s, ri, rf, b, c, nl, n, r0, g->d_dep_ptr.as<int64_t>(), g->d_dep_site.as<int32_t>(),
                               dep_records<T>(g), chi, S, Ifw, gI, gJ, g->d_w.as<double>(), Ibar, Sbar, Cbar);
      }
    }
    vrt::launch_reverse_reduce<T>(s, n, nl, r0, gc, g->d_dirs.as<double>(), g->d_wall.as<uint8_t>(), Ibar, Sbar,
                                  Cbar, acc, acc + nn, acc + 2 * nn, acc + 3 * nn);
  }
  vrt::launch_to_prec<T>(s, nn, acc, o_chi);
  vrt::launch_to_prec<T>(s, nn, acc + nn, o_S);
  vrt::launch_to_prec<T>(s, nn, acc + 2 * nn, o_Ib);
  vrt::launch_to_prec<T>(s, nn, acc + 3 * nn, o_It);
}

// One Lambda iteration without the host read: reset the per-atmosphere
// max-change words, assemble chi and S from S_line, sweep every ray, then Jbar
// and the update of the active atmospheres.
// The library's own chi, S, I_bottom and intensity rows have ld >= nl entries
// (16-byte multiples, so the sweep moves whole vectors); the padding lanes
// carry the continuum and are never read back.
template <typename T>
void enqueue_lambda_step(vrt_grid g, hipStream_t s, vrt_exec ex, int32_t nl, int32_t ld, const double *phi,
                         const double *chi_L, const double *chi_c, const double *B, double eps, double *S_L, T *I,
                         int32_t n_atm, const double *Lbar) {
  // a site's chi and S rows side by side (S = chi + ld, rows 2 ld apart): the
  // sweep's gathers of an upwind site then read one contiguous span
  const int64_t cs = 2 * (int64_t)ld;
  T *chi = g->d_nchi.as<T>(), *S = chi + ld, *Ib = g->d_nIb.as<T>();
  auto *dS = g->d_dS.as<unsigned long long>();
  vrt::launch_zero_u64(s, n_atm, dS);
  vrt::launch_nlte_assemble<T>(s, g->n, nl, ld, cs, phi, chi_L, chi_c, B, S_L, chi, S);
  enqueue_sweep<T>(g, s, ex == VRT_EXEC_GRAPH ? VRT_EXEC_BATCHED : ex, ld, chi, S, Ib, nullptr, I, false, cs);
  vrt::launch_line_update<T>(s, g->n, nl, ld, g->R, I, g->d_w.as<double>(), g->d_wlam.as<double>(), phi, B, eps,
                             S_L, n_atm, g->d_atm_ptr.as<int64_t>(), g->d_active.as<int32_t>(), dS,
                             g->d_jbar.as<double>(), Lbar);
}

// Lambda iteration of n_atm independent atmospheres stored as one grid:
// atmosphere a owns sites [atm_ptr[a], atm_ptr[a+1]). Each is tested for
// convergence on its own and stops updating its S_line once converged, so its
// iterates are those of a solve of that atmosphere alone. hist is
// [max_iter][n_atm] (-1 where an atmosphere had stopped), n_iter [n_atm].
template <typename T>
vrt_status two_level_solve(vrt_grid g, vrt_exec ex, int32_t nl, const double *wlam, const double *phi,
                           const double *chi_L, const double *chi_c, const double *B, double eps, int32_t max_iter,
                           double tol, int32_t accel, double *S_L, int32_t n_atm, const int64_t *atm_ptr,
                           double *hist, int32_t *n_iter) {
  vrt_ctx ctx = g->ctx;
  hipStream_t s = ctx->stream;
  constexpr int32_t per16 = 16 / (int32_t)sizeof(T);
  const int32_t ld = (nl + per16 - 1) / per16 * per16;
  const size_t nn = (size_t)g->n * (size_t)ld;
  ++g->solution_id;  // from here on the last solution's rows may be overwritten
  VRT_HIP(hipStreamSynchronize(s));  // earlier work may still read the buffers replaced below
  // The sign-encoded rows of persistent formal solutions are neither read nor
  // written by the iteration, and the last solution's rows are being replaced:
  // when the device is out of memory for the iteration's scratch, their block
  // goes back to it (a later persistent solution allocates and refills it).
  auto fit = [&](auto &&allocate) {
    try {
      allocate();
    } catch (const vrt::Error &e) {
      if (e.code != VRT_E_NOMEM || !g->d_Isgn.p) throw;
      (void)hipGetLastError();  // the failed allocation is handled here: later launch checks must not see it
      g->d_Isgn.release();
      for (int k = 0; k < 4; ++k) g->sgn_key[k] = 0;
      if (g->last_abs) {
        g->last_I = nullptr;  // the rows it pointed to are gone
        g->last_abs = false;
      }
      allocate();
    }
  };
  T *I = nullptr;
  fit([&] { I = intensity_buffer<T>(g, ld, nullptr); });
  // chi and S rows paired, 2 ld apart; the bottom boundary rows (B) at the same stride
  fit([&] { g->d_nchi.alloc(2 * nn * sizeof(T)); });
  fit([&] { g->d_nIb.alloc(2 * nn * sizeof(T)); });
  g->d_jbar.alloc((size_t)g->n * 8);
  g->d_dS.alloc((size_t)n_atm * 8);
  g->d_atm_ptr.alloc((size_t)(n_atm + 1) * 8);
  g->d_active.alloc((size_t)n_atm * 4 + 4);  // the last word is the partition-check flag
  if (g->h_dS_cap < n_atm) {
    if (g->h_dS) (void)hipHostFree(g->h_dS);
    if (g->h_active) (void)hipHostFree(g->h_active);
    g->h_dS = nullptr;
    g->h_active = nullptr;
    g->h_dS_cap = 0;
    VRT_HIP(hipHostMalloc((void **)&g->h_dS, (size_t)n_atm * 8, hipHostMallocDefault));
    VRT_HIP(hipHostMalloc((void **)&g->h_active, (size_t)n_atm * 4 + 4, hipHostMallocDefault));
    g->h_dS_cap = n_atm;
  }
  g->d_wlam.alloc((size_t)nl * 8);
  VRT_HIP(hipMemcpy(g->d_wlam.p, wlam, (size_t)nl * 8, hipMemcpyHostToDevice));
  VRT_HIP(hipMemcpy(g->d_atm_ptr.p, atm_ptr, (size_t)(n_atm + 1) * 8, hipMemcpyHostToDevice));
  int32_t *active = g->h_active;
  for (int32_t a = 0; a < n_atm; ++a) active[a] = 1;
  active[n_atm] = 0;
  int32_t *d_bad = g->d_active.as<int32_t>() + n_atm;
  VRT_HIP(hipMemcpy(g->d_active.p, active, (size_t)n_atm * 4 + 4, hipMemcpyHostToDevice));
  if (n_atm > 1) {
    vrt::launch_check_partition(s, g->n, g->R, g->d_k1.as<int32_t>(), g->d_k2.as<int32_t>(), n_atm,
                                g->d_atm_ptr.as<int64_t>(), d_bad);
    int32_t bad = 0;
    VRT_HIP(hipMemcpyAsync(&bad, d_bad, 4, hipMemcpyDeviceToHost, s));
    VRT_HIP(hipStreamSynchronize(s));
    if (bad) fail(VRT_E_GRID, "a site reads an upwind neighbour in another atmosphere");
  }
  vrt::launch_broadcast<T>(s, g->n, ld, 2 * (int64_t)ld, B, g->d_nIb.as<T>());
  const double *Lbar = nullptr;
  if (accel) {
    if (g->kind != 0) fail(VRT_E_ARG, "the accelerated iteration needs a Voronoi grid");
    g->d_lbar.alloc((size_t)g->n * 8);
    vrt::launch_line_diag(s, g->n, nl, g->R, g->d_w.as<double>(), g->d_k1.as<int32_t>(), g->d_k2.as<int32_t>(),
                          g->d_w1.as<double>(), g->d_ds1.as<double>(), g->d_ds2.as<double>(), chi_c, chi_L, phi,
                          g->d_wlam.as<double>(), g->d_lbar.as<double>());
    Lbar = g->d_lbar.as<double>();
  }
  const int pexec = ex == VRT_EXEC_PERSISTENT && g->kind == 0 ? 1 : 0;
  const bool use_graph = ex == VRT_EXEC_GRAPH || (ex == VRT_EXEC_PERSISTENT && g->kind != 0);
  if (use_graph) {
    const auto key = std::make_tuple((int)sizeof(T), nl, (const void *)phi, (const void *)chi_L,
                                     (const void *)chi_c, (const void *)B, (const void *)S_L, eps, pexec, n_atm,
                                     (const void *)g->d_atm_ptr.p, (const void *)g->d_active.p,
                                     (const void *)g->d_dS.p, accel ? 1 : 0);
    // the graph also bakes in the scratch pointers, which the allocations above may have moved
    const bool same = g->nlte_graph && g->nlte_key == key && g->nlte_scratch[0] == g->d_nchi.p &&
                      g->nlte_scratch[2] == g->d_nIb.p &&
                      g->nlte_scratch[3] == (const void *)I && g->nlte_scratch[4] == g->d_wlam.p &&
                      g->nlte_scratch[5] == g->d_jbar.p && g->nlte_scratch[6] == (const void *)Lbar;
    if (!same) {
      if (g->nlte_graph) (void)hipGraphExecDestroy(g->nlte_graph);
      g->nlte_graph = nullptr;
      if (!ctx->capture_stream) VRT_HIP(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
      hipStream_t cs = ctx->capture_stream;
      VRT_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      hipGraph_t graph = nullptr;
      try {
        enqueue_lambda_step<T>(g, cs, VRT_EXEC_GRAPH, nl, ld, phi, chi_L, chi_c, B, eps, S_L, I, n_atm, Lbar);
      } catch (...) {
        (void)hipStreamEndCapture(cs, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
      }
      VRT_HIP(hipStreamEndCapture(cs, &graph));
      hipError_t e = hipGraphInstantiate(&g->nlte_graph, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      VRT_HIP(e);
      g->nlte_key = key;
      g->nlte_scratch[0] = g->d_nchi.p;
      g->nlte_scratch[1] = nullptr;
      g->nlte_scratch[2] = g->d_nIb.p;
      g->nlte_scratch[3] = I;
      g->nlte_scratch[4] = g->d_wlam.p;
      g->nlte_scratch[5] = g->d_jbar.p;
      g->nlte_scratch[6] = Lbar;
    }
  }
  for (int32_t a = 0; a < n_atm; ++a) n_iter[a] = 0;
  int32_t n_active = n_atm;
  for (int32_t it = 0; it < max_iter && n_active > 0; ++it) {
    if (use_graph)
      VRT_HIP(hipGraphLaunch(g->nlte_graph, s));
    else
      enqueue_lambda_step<T>(g, s, ex, nl, ld, phi, chi_L, chi_c, B, eps, S_L, I, n_atm, Lbar);
    VRT_HIP(hipMemcpyAsync(g->h_dS, g->d_dS.p, (size_t)n_atm * 8, hipMemcpyDeviceToHost, s));
    VRT_HIP(hipStreamSynchronize(s));
    if (pexec) take_device_error(g, it + 1);
    bool changed = false;
    for (int32_t a = 0; a < n_atm; ++a) {
      double d = -1.0;
      if (active[a]) {
        std::memcpy(&d, g->h_dS + a, 8);
        n_iter[a] = it + 1;
        if (!std::isfinite(d)) {
          if (hist) hist[(size_t)it * n_atm + a] = d;
          fail(VRT_E_NUMERIC, "non-finite source-function change in atmosphere %d at iteration %d", a, it + 1);
        }
        if (d < tol) {
          active[a] = 0;
          --n_active;
          changed = true;
        }
      }
      if (hist) hist[(size_t)it * n_atm + a] = d;
    }
    if (changed && n_active > 0)
      VRT_HIP(hipMemcpyAsync(g->d_active.p, active, (size_t)n_atm * 4, hipMemcpyHostToDevice, s));
  }
  g->last_I = I;
  g->last_abs = false;
  g->last_prec = sizeof(T) == 4 ? VRT_F32 : VRT_F64;
  g->last_nl = nl;
  g->last_ld = ld;
  g->last_own = true;
  ++g->solution_id;
  return n_active == 0 ? VRT_OK : VRT_W_NOT_CONVERGED;
}

// cs: the row stride of chi, S, Ib and It in elements (0: nl)
template <typename T>
void formal_solution(vrt_grid g, vrt_exec ex, int32_t nl, const void *chi_, const void *S_, const void *Ib_,
                     const void *It_, void *J_, void *Ir_, int64_t cs = 0) {
  const T *chi = static_cast<const T *>(chi_), *S = static_cast<const T *>(S_);
  const T *Ib = Ib_ ? static_cast<const T *>(Ib_) : S;
  const T *It = static_cast<const T *>(It_);
  T *J = static_cast<T *>(J_);
  vrt_ctx ctx = g->ctx;
  ++g->solution_id;  // from here on the last solution's rows may be overwritten
  if (ex == VRT_EXEC_PERSISTENT && g->kind != 0) ex = VRT_EXEC_GRAPH;
  // the linear-segment persistent sweep into the library's own rows uses the
  // sign-encoded protocol; rows handed in by the caller keep the stamps
  const bool sign = ex == VRT_EXEC_PERSISTENT && g->segment == 0 && !Ir_;
  T *I = sign ? sign_buffer<T>(g, nl) : intensity_buffer<T>(g, nl, Ir_);
  if (cs == 0) cs = nl;
  if (ex != VRT_EXEC_GRAPH) {
    enqueue_fs<T>(g, ctx->stream, ex, nl, chi, S, Ib, It, J, I, sign, cs);
  } else {
    const vrt_grid_s::GraphKey key{sizeof(T), nl, cs, chi, S, Ib, It, J, I};
    auto it = g->graphs.find(key);
    if (it == g->graphs.end() && g->graphs.size() >= 8) {
      // bounded cache: callers that pass fresh buffers every time would otherwise grow it without end
      for (auto &kv : g->graphs) (void)hipGraphExecDestroy(kv.second);
      g->graphs.clear();
    }
    if (it == g->graphs.end()) {
      if (!ctx->capture_stream) VRT_HIP(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
      hipStream_t cap_s = ctx->capture_stream;
      VRT_HIP(hipStreamBeginCapture(cap_s, hipStreamCaptureModeThreadLocal));
      hipGraph_t graph = nullptr;
      try {
        enqueue_fs<T>(g, cap_s, VRT_EXEC_BATCHED, nl, chi, S, Ib, It, J, I, false, cs);
      } catch (...) {
        (void)hipStreamEndCapture(cap_s, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
      }
      VRT_HIP(hipStreamEndCapture(cap_s, &graph));
      hipGraphExec_t exec = nullptr;
      hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      VRT_HIP(e);
      it = g->graphs.emplace(key, exec).first;
    }
    VRT_HIP(hipGraphLaunch(it->second, ctx->stream));
  }
  g->last_I = I;
  g->last_abs = sign;
  g->last_prec = sizeof(T) == 4 ? VRT_F32 : VRT_F64;
  g->last_nl = nl;
  g->last_ld = nl;
  g->last_own = Ir_ == nullptr;
  ++g->solution_id;
}

bool valid_prec(vrt_prec p) { return p == VRT_F64 || p == VRT_F32; }

// frees a grid whose context is still alive (the context's stream is drained first)
void free_grid(vrt_grid g) {
  (void)hipSetDevice(g->ctx->device);
  (void)hipStreamSynchronize(g->ctx->stream);
  g->drop_graphs();
  if (g->h_dS) (void)hipHostFree(g->h_dS);
  if (g->h_active) (void)hipHostFree(g->h_active);
  delete g;
}

}  // namespace

void vrt_ctx_s::ensure_aux(int k) {
  if (!fork_ev) VRT_HIP(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming));
  while ((int)aux.size() < k) {
    hipStream_t a = nullptr;
    VRT_HIP(hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
    aux.push_back(a);
    hipEvent_t e = nullptr;
    VRT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    join_ev.push_back(e);
  }
}

void vrt_ctx_s::drain_profile() {
  for (auto &t : pending) {
    VRT_HIP(hipEventSynchronize(t.stop));
    float ms = 0.0f;
    VRT_HIP(hipEventElapsedTime(&ms, t.start, t.stop));
    prof_ms[t.kernel] += ms;
    prof_launches[t.kernel] += 1;
    prof_units[t.kernel] += t.units;
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  pending.clear();
}

void vrt_grid_s::drop_graphs() {
  for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
  graphs.clear();
  if (nlte_graph) (void)hipGraphExecDestroy(nlte_graph);
  nlte_graph = nullptr;
}

extern "C" {

const char *vrt_version(void) { return kVersion; }

const char *vrt_status_string(vrt_status s) {
  switch (s) {
    case VRT_OK: return "ok";
    case VRT_W_NOT_CONVERGED: return "not converged";
    case VRT_E_ARG: return "invalid argument";
    case VRT_E_GRID: return "invalid grid";
    case VRT_E_DAG: return "upwind graph is not acyclic";
    case VRT_E_HIP: return "HIP error";
    case VRT_E_NOMEM: return "out of memory";
    case VRT_E_NUMERIC: return "numerical error";
    case VRT_E_STATE: return "call out of order";
    case VRT_E_TIMEOUT: return "device wait timed out";
    default: return "unknown status";
  }
}

vrt_status vrt_validate_voronoi(int64_t n, const double *xyz, const int64_t *nbr_ptr, const int32_t *nbr_idx,
                                const int8_t *nbr_shift, const uint8_t *wall, const double lo[3], const double hi[3],
                                uint32_t periodic_xy, char *msg, int64_t msg_len) {
  try {
    if (!lo || !hi || (n > 0 && !nbr_ptr)) {
      if (msg && msg_len > 0) snprintf(msg, (size_t)msg_len, "null argument");
      return VRT_E_ARG;
    }
    const std::string err = check_voronoi(n, xyz, nbr_ptr, nbr_idx, nbr_shift, wall, lo, hi, periodic_xy != 0);
    if (msg && msg_len > 0) snprintf(msg, (size_t)msg_len, "%s", err.c_str());
    return err.empty() ? VRT_OK : VRT_E_GRID;
  } catch (...) {
    if (msg && msg_len > 0) snprintf(msg, (size_t)msg_len, "host allocation failed");
    return VRT_E_NOMEM;
  }
}

vrt_status vrt_ctx_create(int32_t device, void *stream, vrt_ctx *out) {
  if (!out) return VRT_E_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return VRT_E_ARG;
  auto *c = new (std::nothrow) vrt_ctx_s;
  if (!c) return VRT_E_NOMEM;
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  if (hipSetDevice(device) != hipSuccess || !init_scratch_dev(device)) {
    delete c;
    return VRT_E_HIP;
  }
  *out = c;
  return VRT_OK;
}

void vrt_ctx_destroy(vrt_ctx ctx) {
  if (!ctx) return;
  for (vrt_grid g : ctx->grids) free_grid(g);
  ctx->grids.clear();
  (void)hipSetDevice(ctx->device);
  try {
    ctx->drain_profile();
  } catch (...) {
  }
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  for (hipStream_t a : ctx->aux) (void)hipStreamDestroy(a);
  for (hipEvent_t e : ctx->join_ev) (void)hipEventDestroy(e);
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  delete ctx;
}

const char *vrt_ctx_last_error(vrt_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

vrt_status vrt_ctx_set_stream(vrt_ctx ctx, void *stream) {
  if (!ctx) return VRT_E_ARG;
  return guarded(ctx, [&] {
    ctx->stream = static_cast<hipStream_t>(stream);
    return VRT_OK;
  });
}

vrt_status vrt_ctx_set_profiling(vrt_ctx ctx, int32_t on) {
  if (!ctx) return VRT_E_ARG;
  return guarded(ctx, [&] {
    ctx->profiling = on != 0;
    return VRT_OK;
  });
}

vrt_status vrt_ctx_profile(vrt_ctx ctx, int32_t kernel, double *ms, int64_t *launches, int64_t *units) {
  if (!ctx) return VRT_E_ARG;
  return guarded(ctx, [&] {
    if (kernel < 0 || kernel > 2) fail(VRT_E_ARG, "kernel class %d not in 0..2", kernel);
    ctx->drain_profile();
    if (ms) *ms = ctx->prof_ms[kernel];
    if (launches) *launches = ctx->prof_launches[kernel];
    if (units) *units = ctx->prof_units[kernel];
    return VRT_OK;
  });
}

vrt_status vrt_ctx_profile_reset(vrt_ctx ctx) {
  if (!ctx) return VRT_E_ARG;
  return guarded(ctx, [&] {
    ctx->drain_profile();
    for (int k = 0; k < 3; ++k) {
      ctx->prof_ms[k] = 0.0;
      ctx->prof_launches[k] = 0;
      ctx->prof_units[k] = 0;
    }
    return VRT_OK;
  });
}

vrt_status vrt_ctx_synchronize(vrt_ctx ctx) {
  if (!ctx) return VRT_E_ARG;
  return guarded(ctx, [&] {
    VRT_HIP(hipStreamSynchronize(ctx->stream));
    return VRT_OK;
  });
}

vrt_status vrt_grid_create_voronoi(vrt_ctx ctx, int64_t n, const double *xyz, const int64_t *nbr_ptr,
                                   const int32_t *nbr_idx, const int8_t *nbr_shift, const uint8_t *wall,
                                   const double lo[3], const double hi[3], uint32_t periodic_xy, vrt_grid *out) {
  if (!ctx || !out) return VRT_E_ARG;
  *out = nullptr;
  return guarded(ctx, [&] {
    if (!lo || !hi || n < 0 || (n > 0 && (!xyz || !nbr_ptr || !wall))) fail(VRT_E_ARG, "null argument or n < 0");
    const std::string err = check_voronoi(n, xyz, nbr_ptr, nbr_idx, nbr_shift, wall, lo, hi, periodic_xy != 0);
    if (!err.empty()) throw Error(VRT_E_GRID, err);
    std::unique_ptr<vrt_grid_s> g(new vrt_grid_s);
    g->ctx = ctx;
    g->kind = 0;
    g->n = n;
    g->m = n > 0 ? nbr_ptr[n] : 0;
    g->periodic = periodic_xy != 0;
    for (int d = 0; d < 3; ++d) {
      g->lo[d] = lo[d];
      g->hi[d] = hi[d];
    }
    hipStream_t s = ctx->stream;
    std::vector<int8_t> zero;
    upload(g->d_xyz, xyz, (size_t)n * 3, s);
    upload(g->d_ptr, nbr_ptr, (size_t)n + 1, s);
    upload(g->d_idx, nbr_idx, (size_t)g->m, s);
    if (nbr_shift) {
      upload(g->d_shift, nbr_shift, (size_t)g->m * 2, s);
    } else {
      zero.assign((size_t)g->m * 2, 0);
      upload(g->d_shift, zero.data(), zero.size(), s);
    }
    upload(g->d_wall, wall, (size_t)n, s);
    g->h_wall.assign(wall, wall + n);
    g->h_xyz.assign(xyz, xyz + 3 * n);
    VRT_HIP(hipStreamSynchronize(s));
    ctx->grids.insert(g.get());
    *out = g.release();
    return VRT_OK;
  });
}

vrt_status vrt_grid_create_regular(vrt_ctx ctx, int32_t nx, int32_t ny, int32_t nz, double dx, double dy,
                                   const double *z, vrt_grid *out) {
  if (!ctx || !out) return VRT_E_ARG;
  *out = nullptr;
  return guarded(ctx, [&] {
    if (nx <= 0 || ny <= 0 || nz <= 0 || !z || !(dx > 0) || !(dy > 0)) fail(VRT_E_ARG, "bad regular grid size");
    if ((int64_t)nx * ny * nz >= (int64_t(1) << 31)) fail(VRT_E_ARG, "more than 2^31 - 1 points");
    for (int32_t k = 1; k < nz; ++k)
      if (!(z[k] > z[k - 1])) fail(VRT_E_GRID, "z must be strictly increasing (index %d)", k);
    std::unique_ptr<vrt_grid_s> g(new vrt_grid_s);
    g->ctx = ctx;
    g->kind = 1;
    g->nx = nx;
    g->ny = ny;
    g->nz = nz;
    g->dx = dx;
    g->dy = dy;
    g->n = (int64_t)nx * ny * nz;
    g->h_z.assign(z, z + nz);
    upload(g->d_z, z, (size_t)nz, ctx->stream);
    VRT_HIP(hipStreamSynchronize(ctx->stream));
    ctx->grids.insert(g.get());
    *out = g.release();
    return VRT_OK;
  });
}

void vrt_grid_destroy(vrt_grid g) {
  if (!g) return;
  g->ctx->grids.erase(g);
  free_grid(g);
}

vrt_status vrt_grid_set_rays(vrt_grid g, int32_t n_rays, const double *dir, const double *w, double r_exp) {
  if (!g) return VRT_E_ARG;
  return guarded(g->ctx, [&] {
    if (n_rays <= 0 || !dir || !w || !std::isfinite(r_exp) || r_exp <= 0)
      fail(VRT_E_ARG, "need n_rays > 0, directions, weights and a positive exponent");
    double sum = 0.0;
    for (int32_t r = 0; r < n_rays; ++r) {
      const double a = dir[3 * r], b = dir[3 * r + 1], c = dir[3 * r + 2];
      const double nrm = std::sqrt(a * a + b * b + c * c);
      if (!(std::fabs(nrm - 1.0) < 1e-12)) fail(VRT_E_ARG, "direction %d is not a unit vector", r);
      if (!(c != 0.0)) fail(VRT_E_ARG, "direction %d is horizontal", r);
      if (!(w[r] > 0.0) || !std::isfinite(w[r])) fail(VRT_E_ARG, "weight %d is not positive", r);
      sum += w[r];
    }
    if (!(std::fabs(sum - 1.0) < 1e-12)) fail(VRT_E_ARG, "ray weights sum to %.17g, not 1", sum);
    g->drop_graphs();
    g->persist_items.clear();
    g->reverse_items.clear();
    g->d_flags.release();
    g->d_epoch.release();
    g->deps_built = false;
    g->R = n_rays;
    g->r_exp = r_exp;
    g->h_dirs.assign(dir, dir + 3 * (size_t)n_rays);
    g->h_w.assign(w, w + n_rays);
    upload(g->d_dirs, dir, 3 * (size_t)n_rays, g->ctx->stream);
    upload(g->d_w, w, (size_t)n_rays, g->ctx->stream);
    g->d_Iscr.release();
    g->d_Isgn.release();
    for (int k = 0; k < 4; ++k) g->sgn_key[k] = 0;
    g->last_I = nullptr;  // the rows it pointed to are gone
    g->last_abs = false;
    ++g->solution_id;
    if (g->kind == 0) {
      set_rays_voronoi(g);
    } else {
      g->n_steps = g->nz;
      g->n_levels.assign((size_t)n_rays, g->nz);
    }
    build_emergent_index(g);
    return VRT_OK;
  });
}

vrt_status vrt_grid_tune(vrt_grid g, int32_t knob, int64_t value) {
  if (!g) return VRT_E_ARG;
  return guarded(g->ctx, [&] {
    if (knob == VRT_TUNE_RECORD_ORDER) {
      if (value != 0 && value != 1) fail(VRT_E_ARG, "record order must be 0 or 1");
      g->record_order = (int)value;
    } else if (knob == VRT_TUNE_XCD_CHUNKS) {
      if (value < 0 || value > 64) fail(VRT_E_ARG, "XCD chunk count must be in 0..64");
      g->xcd_chunks = (int)value;
    } else if (knob == VRT_TUNE_RAY_AFFINITY) {
      if (value != 0 && value != 1) fail(VRT_E_ARG, "ray affinity must be 0 or 1");
      g->ray_affinity = (int)value;
    } else if (knob == VRT_TUNE_CHAINS) {
      if (value < 1 || value > 8) fail(VRT_E_ARG, "chain count must be in 1..8");
      g->chains = (int)value;
    } else if (knob == VRT_TUNE_RAY_GROUPS) {
      if (value < 1 || value > 64) fail(VRT_E_ARG, "ray groups must be in 1..64");
      g->ray_groups = (int)value;
    } else if (knob == VRT_TUNE_INTERLEAVE) {
      if (value < 0 || value > 2) fail(VRT_E_ARG, "interleave must be 0, 1 or 2");
      g->interleave = (int)value;
      if (g->interleave && g->kind == 0 && g->R > 0 && g->interleaved_built != g->interleave) build_interleaved(g);
    } else if (knob == VRT_TUNE_SEGMENT) {
      if (value != 0 && value != 1) fail(VRT_E_ARG, "segment must be 0 (linear) or 1 (quadratic Bezier)");
      if (value == 1 && g->kind != 0) fail(VRT_E_ARG, "the quadratic segment needs a Voronoi grid");
      g->segment = (int)value;
      if (g->segment && g->R > 0 && !g->down_built) build_downwind(g);
    } else if (knob == VRT_TUNE_REVERSE_PERSISTENT) {
      if (value != 0 && value != 1) fail(VRT_E_ARG, "reverse persistent must be 0 or 1");
      g->reverse_persistent = (int)value;
    } else if (knob == VRT_TUNE_PIPELINE) {
      if (value != 0 && value != 2 && value != 4 && value != 8) fail(VRT_E_ARG, "pipeline depth must be 0, 2, 4 or 8");
      g->pipe = (int)value;
    } else if (knob == VRT_TUNE_SHARED_LEVELS) {
      if (value != 0 && value != 1) fail(VRT_E_ARG, "shared levels must be 0 or 1");
      if (g->kind == 0 && (int)value != g->shared_levels) {
        g->shared_levels = (int)value;
        if (g->R > 0) {
          // new level steps: the item tables and every schedule-derived table go
          g->drop_graphs();
          g->persist_items.clear();
          g->reverse_items.clear();
          set_rays_voronoi(g);
        }
      }
    } else if (knob == VRT_TUNE_REGULAR_TILE) {
      if (value < 0 || value > 2) fail(VRT_E_ARG, "regular tiling must be 0, 1 or 2");
      g->regular_tiled = (int)value;
    } else if (knob == VRT_TUNE_LANE_BYTES) {
      if (value != 16 && value != 32) fail(VRT_E_ARG, "lane bytes must be 16 or 32");
      g->lane_bytes = (int)value;
    } else if (knob == VRT_TUNE_SPIN_CAP) {
      if (value < 0) fail(VRT_E_ARG, "spin cap must be non-negative");
      g->spin_cap = value;
    } else if (knob == VRT_TUNE_PERSIST_BLOCKS) {
      if (value < 0 || value > (int64_t(1) << 20)) fail(VRT_E_ARG, "bad persistent block cap");
      g->persist_max_blocks = (int32_t)value;
    } else {
      fail(VRT_E_ARG, "unknown tuning knob %d", knob);
    }
    g->drop_graphs();
    return VRT_OK;
  });
}

vrt_status vrt_grid_autotune(vrt_grid g, vrt_prec prec, int32_t n_lambda, const void *chi, const void *S,
                             const void *I_bottom, const void *I_top, void *J, void *I_rays, int32_t reps, char *report,
                             int64_t report_len) {
  if (!g) return VRT_E_ARG;
  return guarded(g->ctx, [&] {
    if (!valid_prec(prec) || n_lambda <= 0 || reps <= 0) fail(VRT_E_ARG, "bad autotune arguments");
    if (g->R == 0) fail(VRT_E_STATE, "rays not set");
    if (g->segment) fail(VRT_E_ARG, "the autotuner times the linear sweep's layouts");
    if (g->n == 0) return VRT_OK;
    hipStream_t s = g->ctx->stream;
    hipEvent_t e0, e1;
    VRT_HIP(hipEventCreate(&e0));
    VRT_HIP(hipEventCreate(&e1));
    if (g->kind != 0) {
      // regular grid: the graph-launched plane steps with the row kernel and
      // with the LDS-tiled kernel
      std::string rep = "{\"candidates\": [";
      double best = 1e300;
      int best_tile = g->regular_tiled == 1 ? 1 : 0;
      for (int tile = 0; tile <= 1; ++tile) {
        g->regular_tiled = tile;
        g->drop_graphs();
        auto run = [&] {
          if (prec == VRT_F32)
            formal_solution<float>(g, VRT_EXEC_GRAPH, n_lambda, chi, S, I_bottom, I_top, J, I_rays);
          else
            formal_solution<double>(g, VRT_EXEC_GRAPH, n_lambda, chi, S, I_bottom, I_top, J, I_rays);
        };
        run();  // capture + warm-up
        VRT_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) run();
        VRT_HIP(hipEventRecord(e1, s));
        VRT_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        VRT_HIP(hipEventElapsedTime(&ms, e0, e1));
        const double mean = ms / reps;
        char buf[160];
        snprintf(buf, sizeof buf, "%s{\"exec\": \"graph\", \"regular_tile\": %d, \"ms\": %.5f}", tile ? ", " : "",
                 tile, mean);
        rep += buf;
        if (mean < best) {
          best = mean;
          best_tile = tile;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      g->regular_tiled = best_tile;
      g->tuned_exec = VRT_EXEC_GRAPH;
      g->drop_graphs();
      char buf[160];
      snprintf(buf, sizeof buf, "], \"chosen\": {\"exec\": \"graph\", \"regular_tile\": %d, \"ms\": %.5f}}", best_tile,
               best);
      rep += buf;
      if (report && report_len > 0) snprintf(report, (size_t)report_len, "%s", rep.c_str());
      return VRT_OK;
    }
    struct Cand {
      int xcd, aff, lb, il, pipe, exec;
    };
    struct Setting {
      int order, shared, xcd, aff, lb, il, pipe, exec;
    };
    // graph-launched level steps under die chunks x ray affinity x lane bytes
    // x interleaved copy x pipeline depth, and the persistent sweep (whose
    // launch ignores those knobs), for each record layout: per-ray levels in
    // site order and in Morton order, and levels shared by the rays of one
    // azimuth (Morton order, the layouts that pay there). Split chains are not
    // candidates: kernels on separate queues were measured not to overlap. The
    // interleaved copies sort every step across rays whatever the record order,
    // so they are timed under the Morton order only; they are built on the
    // host, up to 2^28 records.
    const int G = VRT_EXEC_GRAPH, P = VRT_EXEC_PERSISTENT;
    static const Cand cands[] = {{0, 0, 16, 0, 0, G}, {8, 0, 16, 0, 0, G}, {0, 1, 16, 0, 0, G}, {8, 0, 32, 0, 0, G},
                                 {0, 1, 32, 0, 0, G}, {8, 0, 16, 0, 2, G}, {8, 0, 16, 0, 4, G}, {8, 0, 16, 1, 0, G},
                                 {0, 0, 16, 1, 0, G}, {8, 0, 16, 1, 2, G}, {8, 0, 16, 2, 0, G}, {8, 0, 16, 2, 2, G},
                                 {8, 0, 16, 0, 0, P}};
    static const Cand shared_cands[] = {{8, 0, 16, 0, 2, G}, {8, 0, 16, 1, 2, G}, {8, 0, 16, 2, 0, G},
                                        {8, 0, 16, 2, 2, G}, {8, 0, 16, 0, 0, P}, {8, 0, 16, 1, 0, P},
                                        {8, 0, 16, 2, 0, P}};
    struct Layout {
      int order, shared;
      const Cand *c;
      size_t nc;
    };
    const Layout layouts[] = {{0, 0, cands, sizeof cands / sizeof cands[0]},
                              {1, 0, cands, sizeof cands / sizeof cands[0]},
                              {1, 1, shared_cands, sizeof shared_cands / sizeof shared_cands[0]}};
    std::string rep = "{\"candidates\": [";
    double best = 1e300;
    Setting bs{g->record_order, g->shared_levels, g->xcd_chunks, g->ray_affinity, g->lane_bytes, g->interleave,
               g->pipe, g->tuned_exec};
    g->chains = 1;
    bool first = true;
    auto fmt = [](int exec) { return exec == VRT_EXEC_PERSISTENT ? "persistent" : "graph"; };
    for (const Layout &ly : layouts) {
      if (ly.order != g->record_order || ly.shared != g->shared_levels || first) {
        g->record_order = ly.order;
        g->shared_levels = ly.shared;
        g->interleave = 0;
        set_rays_voronoi(g);
      }
      for (size_t ci = 0; ci < ly.nc; ++ci) {
        const Cand &cd = ly.c[ci];
        const int order = ly.order;
        if (cd.il && (order != 1 || g->n_rec > (int64_t(1) << 28))) continue;
        if (cd.exec == P && g->segment) continue;
        g->xcd_chunks = cd.xcd;
        g->ray_affinity = cd.aff;
        g->lane_bytes = cd.lb;
        g->interleave = cd.il;
        g->pipe = cd.pipe;
        if (cd.il && g->interleaved_built != cd.il) build_interleaved(g);
        g->drop_graphs();
        auto run = [&] {
          if (prec == VRT_F32)
            formal_solution<float>(g, (vrt_exec)cd.exec, n_lambda, chi, S, I_bottom, I_top, J, I_rays);
          else
            formal_solution<double>(g, (vrt_exec)cd.exec, n_lambda, chi, S, I_bottom, I_top, J, I_rays);
        };
        double mean = -1.0;
        try {
          run();  // capture + warm-up
          VRT_HIP(hipEventRecord(e0, s));
          for (int r = 0; r < reps; ++r) run();
          VRT_HIP(hipEventRecord(e1, s));
          VRT_HIP(hipEventSynchronize(e1));
          if (cd.exec == P) take_device_error(g, 0);
          float ms = 0.0f;
          VRT_HIP(hipEventElapsedTime(&ms, e0, e1));
          mean = ms / reps;
        } catch (const Error &e) {
          if (e.code == VRT_E_HIP || e.code == VRT_E_NOMEM) throw;
          VRT_HIP(hipStreamSynchronize(s));
          take_device_error(g, 0);  // rethrows a pending device error as its own status
        }
        char buf[288], msb[32];
        if (mean >= 0.0) snprintf(msb, sizeof msb, "%.5f", mean);
        else snprintf(msb, sizeof msb, "null");
        snprintf(buf, sizeof buf,
                 "%s{\"exec\": \"%s\", \"record_order\": %d, \"shared_levels\": %d, \"xcd_chunks\": %d, "
                 "\"ray_affinity\": %d, \"lane_bytes\": %d, \"interleave\": %d, \"pipeline\": %d, \"ms\": %s}",
                 first ? "" : ", ", fmt(cd.exec), order, ly.shared, cd.xcd, cd.aff, cd.lb, cd.il, cd.pipe, msb);
        rep += buf;
        first = false;
        if (mean >= 0.0 && mean < best) {
          best = mean;
          bs = Setting{order, ly.shared, cd.xcd, cd.aff, cd.lb, cd.il, cd.pipe, cd.exec};
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g->chains = 1;  // every candidate was timed with one launch chain
    g->interleave = 0;
    if (bs.order != g->record_order || bs.shared != g->shared_levels) {
      g->record_order = bs.order;
      g->shared_levels = bs.shared;
      set_rays_voronoi(g);
    }
    g->xcd_chunks = bs.xcd;
    g->ray_affinity = bs.aff;
    g->lane_bytes = bs.lb;
    g->interleave = bs.il;
    g->pipe = bs.pipe;
    g->tuned_exec = bs.exec;
    if (bs.il && g->interleaved_built != bs.il) build_interleaved(g);
    g->drop_graphs();
    // the sign-encoded rows the persistent candidates used: when the persistent
    // sweep is not the choice, their block goes back to the device (a later
    // persistent solution allocates and refills it)
    if (bs.exec != VRT_EXEC_PERSISTENT && g->d_Isgn.p) {
      VRT_HIP(hipStreamSynchronize(s));
      g->d_Isgn.release();
      for (int k = 0; k < 4; ++k) g->sgn_key[k] = 0;
      if (g->last_abs) {
        g->last_I = nullptr;  // the rows it pointed to are gone
        g->last_abs = false;
      }
    }
    char buf[352];
    snprintf(buf, sizeof buf,
             "], \"chosen\": {\"exec\": \"%s\", \"record_order\": %d, \"shared_levels\": %d, \"xcd_chunks\": %d, "
             "\"ray_affinity\": %d, \"lane_bytes\": %d, \"interleave\": %d, \"pipeline\": %d, \"ms\": %.5f}}",
             fmt(bs.exec), bs.order, bs.shared, bs.xcd, bs.aff, bs.lb, bs.il, bs.pipe, best);
    rep += buf;
    if (report && report_len > 0) snprintf(report, (size_t)report_len, "%s", rep.c_str());
    return VRT_OK;
  });
}

vrt_status vrt_grid_info(vrt_grid g, int64_t *n_sites, int32_t *n_rays, int32_t *max_levels, int64_t *n_fallback) {
  if (!g) return VRT_E_ARG;
  if (n_sites) *n_sites = g->n;
  if (n_rays) *n_rays = g->R;
  if (max_levels) *max_levels = g->n_steps;
  if (n_fallback) *n_fallback = g->n_fallback;
  return VRT_OK;
}

vrt_status vrt_grid_schedule(vrt_grid g, int32_t ray, int32_t *k1, int32_t *k2, double *w1, double *ds1, double *ds2,
                             int32_t *level, int32_t *order, int32_t *level_ptr, int32_t *n_levels) {
  if (!g) return VRT_E_ARG;
  return guarded(g->ctx, [&] {
    if (g->kind != 0) fail(VRT_E_ARG, "schedules exist on Voronoi grids only");
    if (g->R == 0) fail(VRT_E_STATE, "rays not set");
    if (ray < 0 || ray >= g->R) fail(VRT_E_ARG, "ray %d out of range", ray);
    hipStream_t s = g->ctx->stream;
    const size_t off = (size_t)ray * (size_t)g->n;
    auto dl = [&](void *h, const DevBuf &d, size_t esz) {
      if (h && g->n) VRT_HIP(hipMemcpyAsync(h, (const char *)d.p + off * esz, (size_t)g->n * esz, hipMemcpyDeviceToHost, s));
    };
    dl(k1, g->d_k1, 4);
    dl(k2, g->d_k2, 4);
    dl(w1, g->d_w1, 8);
    dl(ds1, g->d_ds1, 8);
    dl(ds2, g->d_ds2, 8);
    dl(level, g->d_level, 4);
    dl(order, g->d_order, 4);
    VRT_HIP(hipStreamSynchronize(s));
    const auto &lp = g->level_ptr[(size_t)ray];
    if (level_ptr) std::copy(lp.begin(), lp.end(), level_ptr);
    if (n_levels) *n_levels = g->n_levels[(size_t)ray];
    return VRT_OK;
  });
}

vrt_status vrt_lte_continuum_ld(vrt_grid g, vrt_prec prec, int32_t n_lambda, int64_t ld_src, const double *lambda_m,
                                double kappa0, const double *T, const double *rho, void *chi, void *S) {
  if (!g) return VRT_E_ARG;
  return guarded(g->ctx, [&] {
    if (!valid_prec(prec) || n_lambda <= 0 || !lambda_m || !(g->n == 0 || (T && rho && chi && S)))
      fail(VRT_E_ARG, "bad LTE arguments");
    if (ld_src < n_lambda) fail(VRT_E_ARG, "ld_src %lld is below n_lambda %d", (long long)ld_src, n_lambda);
    for (int32_t l = 0; l < n_lambda; ++l)
      if (!(lambda_m[l] > 0.0)) fail(VRT_E_ARG, "wavelength %d is not positive", l);
    hipStream_t s = g->ctx->stream;
    // the wavelength table is cached on the device; a new table waits for
    // earlier work that may still read the old one, then is copied synchronously
    if (g->h_lam.size() != (size_t)n_lambda || !std::equal(g->h_lam.begin(), g->h_lam.end(), lambda_m)) {
      VRT_HIP(hipStreamSynchronize(s));
      g->d_lam.alloc((size_t)n_lambda * sizeof(double));
      VRT_HIP(hipMemcpy(g->d_lam.p, lambda_m, (size_t)n_lambda * sizeof(double), hipMemcpyHostToDevice));
      g->h_lam.assign(lambda_m, lambda_m + n_lambda);
    }
    if (prec == VRT_F32)
      vrt::launch_lte<float>(s, g->n, n_lambda, ld_src, g->d_lam.as<double>(), kappa0, T, rho,
                             static_cast<float *>(chi), static_cast<float *>(S));
    else
      vrt::launch_lte<double>(s, g->n, n_lambda, ld_src, g->d_lam.as<double>(), kappa0, T, rho,
                              static_cast<double *>(chi), static_cast<double *>(S));
    return VRT_OK;
  });
}

vrt_status vrt_lte_continuum(vrt_grid g, vrt_prec prec, int32_t n_lambda, const double *lambda_m, double kappa0,
                             const double *T, const double *rho, void *chi, void *S) {
  return vrt_lte_continuum_ld(g, prec, n_lambda, n_lambda, lambda_m, kappa0, T, rho, chi, S);
}

vrt_status vrt_formal_solution_ld(vrt_grid g, vrt_prec prec, vrt_exec exec, int32_t n_lambda, int64_t ld_src,
                                  const void *chi, const void *S, const void *I_bottom, const void *I_top, void *J,
                                  void *I_rays) {
  if (!g) return VRT_E_ARG;
  return guarded(g->ctx, [&] {
    if (exec == VRT_EXEC_AUTO) exec = (vrt_exec)g->tuned_exec;
    if (!valid_prec(prec) || (exec != VRT_EXEC_PLAIN && exec != VRT_EXEC_BATCHED && exec != VRT_EXEC_GRAPH &&
                              exec != VRT_EXEC_PERSISTENT))
      fail(VRT_E_ARG, "bad precision or execution mode");
    if (n_lambda <= 0) fail(VRT_E_ARG, "n_lambda must be positive");
    if (ld_src < n_lambda) fail(VRT_E_ARG, "ld_src %lld is below n_lambda %d", (long long)ld_src, n_lambda);
    if (g->kind != 0 && ld_src != n_lambda)
      fail(VRT_E_ARG, "a regular grid takes input rows of n_lambda entries (ld_src = n_lambda)");
    if (g->R == 0) fail(VRT_E_STATE, "rays not set");
    if (g->n > 0 && (!chi || !S || !J)) fail(VRT_E_ARG, "chi, S and J are required");
    if (g->n == 0) return VRT_OK;
    if (prec == VRT_F32)
      formal_solution<float>(g, exec, n_lambda, chi, S, I_bottom, I_top, J, I_rays, ld_src);
    else
      formal_solution<double>(g, exec, n_lambda, chi, S, I_bottom, I_top, J, I_rays, ld_src);
    return VRT_OK;
  });
}

vrt_status vrt_formal_solution(vrt_grid g, vrt_prec prec, vrt_exec exec, int32_t n_lambda, const void *chi,
                               const void *S, const void *I_bottom, const void *I_top, void *J, void *I_rays) {
  return vrt_formal_solution_ld(g, prec, exec, n_lambda, n_lambda, chi, S, I_bottom, I_top, J, I_rays);
}

vrt_status vrt_formal_solution_noalloc(vrt_grid g, vrt_prec prec, int32_t n_lambda, const void *chi, const void *S,
                                       const void *I_bottom, const void *I_top, void *J) {
  if (!g) return VRT_E_ARG;
  return guarded(g->ctx, [&] {
    if (!valid_prec(prec)) fail(VRT_E_ARG, "bad precision");
    if (n_lambda <= 0) fail(VRT_E_ARG, "n_lambda must be positive");
    if (g->R == 0) fail(VRT_E_STATE, "rays not set");
    if (g->n > 0 && (!chi || !S || !J)) fail(VRT_E_ARG, "chi, S and J are required");
    if (g->n == 0) return VRT_OK;
    const size_t elem = prec == VRT_F32 ? 4 : 8;
    const size_t need = (size_t)g->R * (size_t)g->n * (size_t)n_lambda * elem;
    if (need > kNoAllocScratchBytes)
      fail(VRT_E_ARG, "the intensities of %d rays x %lld sites x %d wavelengths take %zu bytes; the "
                      "no-allocation entry point holds %zu (use vrt_formal_solution)",
           g->R, (long long)g->n, n_lambda, need, kNoAllocScratchBytes);
    if (g->kind == 0 && g->chains > 1 && !g->ray_affinity)
      fail(VRT_E_ARG, "split launch chains create streams: set VRT_TUNE_CHAINS to 1 for this entry point");
    void *base = scratch_dev(g->ctx->device);
    if (!base) fail(VRT_E_STATE, "no scratch address for device %d", g->ctx->device);
    // the level-step sweeps and the J quadrature of vrt_formal_solution in the
    // batched mode, eagerly and without timing events, with the intensities in
    // the static scratch
    vrt_ctx ctx = g->ctx;
    const bool prof = ctx->profiling;
    ctx->profiling = false;
    try {
      if (prec == VRT_F32) {
        const float *c = static_cast<const float *>(chi), *s = static_cast<const float *>(S);
        enqueue_fs<float>(g, ctx->stream, VRT_EXEC_BATCHED, n_lambda, c, s,
                          I_bottom ? static_cast<const float *>(I_bottom) : s, static_cast<const float *>(I_top),
                          static_cast<float *>(J), static_cast<float *>(base));
      } else {
        const double *c = static_cast<const double *>(chi), *s = static_cast<const double *>(S);
        enqueue_fs<double>(g, ctx->stream, VRT_EXEC_BATCHED, n_lambda, c, s,
                           I_bottom ? static_cast<const double *>(I_bottom) : s, static_cast<const double *>(I_top),
                           static_cast<double *>(J), static_cast<double *>(base));
      }
    } catch (...) {
      ctx->profiling = prof;
      throw;
    }
    ctx->profiling = prof;
    // the rows stay in scratch that every call on this device shares: no
    // later gather may read them as this grid's last solution
    g->last_I = nullptr;
    g->last_abs = false;
    ++g->solution_id;
    return VRT_OK;
  });
}

static vrt_status two_level_entry(vrt_grid g, vrt_prec prec, vrt_exec exec, int32_t n_lambda, const double *wlam,
                                  const double *phi, const double *chi_line, const double *chi_cont, const double *B,
                                  double eps, int32_t max_iter, double tol, int32_t accel, double *S_line,
                                  int32_t n_atm, const int64_t *atm_ptr, double *dS_hist, int32_t *n_iter) {
  if (!valid_prec(prec) || n_lambda <= 0 || !wlam || max_iter < 0 || !(tol >= 0.0) || !(eps >= 0.0 && eps <= 1.0))
    fail(VRT_E_ARG, "bad two-level arguments");
  if (exec == VRT_EXEC_AUTO) exec = (vrt_exec)g->tuned_exec;
  if (exec != VRT_EXEC_PLAIN && exec != VRT_EXEC_BATCHED && exec != VRT_EXEC_GRAPH && exec != VRT_EXEC_PERSISTENT)
    fail(VRT_E_ARG, "bad execution mode");
  if (n_atm <= 0 || !atm_ptr || !n_iter) fail(VRT_E_ARG, "bad atmosphere partition");
  if (atm_ptr[0] != 0 || atm_ptr[n_atm] != g->n) fail(VRT_E_ARG, "atmosphere offsets must run from 0 to n");
  for (int32_t a = 0; a < n_atm; ++a)
    if (atm_ptr[a + 1] < atm_ptr[a]) fail(VRT_E_ARG, "atmosphere offsets must not decrease");
  if (n_atm > 1 && g->kind != 0) fail(VRT_E_ARG, "several atmospheres need a Voronoi grid");
  if (g->R == 0) fail(VRT_E_STATE, "rays not set");
  for (int32_t a = 0; a < n_atm; ++a) n_iter[a] = 0;
  if (g->n == 0 || max_iter == 0) return max_iter == 0 ? VRT_W_NOT_CONVERGED : VRT_OK;
  if (!phi || !chi_line || !chi_cont || !B || !S_line) fail(VRT_E_ARG, "null device array");
  if (accel != 0 && accel != 1) fail(VRT_E_ARG, "accel must be 0 or 1");
  if (g->segment && accel) fail(VRT_E_ARG, "the quadratic segment runs the plain (unaccelerated) iteration");
  if (prec == VRT_F32)
    return two_level_solve<float>(g, exec, n_lambda, wlam, phi, chi_line, chi_cont, B, eps, max_iter, tol, accel,
                                  S_line, n_atm, atm_ptr, dS_hist, n_iter);
  return two_level_solve<double>(g, exec, n_lambda, wlam, phi, chi_line, chi_cont, B, eps, max_iter, tol, accel,
                                 S_line, n_atm, atm_ptr, dS_hist, n_iter);
}

vrt_status vrt_two_level_solve(vrt_grid g, vrt_prec prec, vrt_exec exec, int32_t n_lambda, const double *wlam,
                               const double *phi, const double *chi_line, const double *chi_cont, const double *B,
                               double eps, int32_t max_iter, double tol, int32_t accel, double *S_line,
                               double *dS_hist, int32_t *n_iter) {
  if (!g) return VRT_E_ARG;
  return guarded(g->ctx, [&]() -> vrt_status {
    const int64_t ptr[2] = {0, g->n};
    int32_t it = 0;
    vrt_status st = VRT_OK;
    try {
      st = two_level_entry(g, prec, exec, n_lambda, wlam, phi, chi_line, chi_cont, B, eps, max_iter, tol, accel,
                           S_line, 1, ptr, dS_hist, &it);
    } catch (...) {
      if (n_iter) *n_iter = it;
      throw;
    }
    if (n_iter) *n_iter = it;
    return st;
  });
}

vrt_status vrt_two_level_solve_batched(vrt_grid g, vrt_prec prec, vrt_exec exec, int32_t n_lambda,
                                       const double *wlam, const double *phi, const double *chi_line,
                                       const double *chi_cont, const double *B, double eps, int32_t max_iter,
                                       double tol, int32_t accel, double *S_line, int32_t n_atm,
                                       const int64_t *atm_ptr, double *dS_hist, int32_t *n_iter) {
  if (!g) return VRT_E_ARG;
  return guarded(g->ctx, [&]() -> vrt_status {
    return two_level_entry(g, prec, exec, n_lambda, wlam, phi, chi_line, chi_cont, B, eps, max_iter, tol, accel,
                           S_line, n_atm, atm_ptr, dS_hist, n_iter);
  });
}

vrt_status vrt_formal_solution_vjp(vrt_grid g, vrt_prec prec, int32_t n_lambda, const void *chi, const void *S,
                                   const void *I_bottom, const void *I_top, const void *I_rays, const void *dL_dI,
                                   const void *dL_dJ, void *dL_dchi, void *dL_dS, void *dL_dIbottom, void *dL_dItop,
                                   int32_t ray_group, int32_t checkpoint_levels) {
  if (!g) return VRT_E_ARG;
  return guarded(g->ctx, [&] {
    if (!valid_prec(prec) || n_lambda <= 0 || ray_group < 0 || checkpoint_levels < 0)
      fail(VRT_E_ARG, "bad precision, n_lambda, ray group or checkpoint interval");
    if (g->kind != 0) fail(VRT_E_ARG, "the reverse sweep exists for Voronoi grids only");
    if (g->segment) fail(VRT_E_ARG, "the reverse sweep differentiates the linear segment only");
    if (g->R == 0) fail(VRT_E_STATE, "rays not set");
    if (g->n == 0) return VRT_OK;
    if (!chi || !S) fail(VRT_E_ARG, "chi and S are required");
    if (!dL_dI && !dL_dJ) fail(VRT_E_ARG, "give dL_dI, dL_dJ or both");
    if (prec == VRT_F32) {
      using T = float;
      const T *ib = I_bottom ? (const T *)I_bottom : (const T *)S;
      formal_solution_vjp<T>(g, n_lambda, (const T *)chi, (const T *)S, ib, (const T *)I_top, (const T *)I_rays,
                             (const T *)dL_dI, (const T *)dL_dJ, (T *)dL_dchi, (T *)dL_dS, (T *)dL_dIbottom,
                             (T *)dL_dItop, ray_group, checkpoint_levels);
    } else {
      using T = double;
      const T *ib = I_bottom ? (const T *)I_bottom : (const T *)S;
      formal_solution_vjp<T>(g, n_lambda, (const T *)chi, (const T *)S, ib, (const T *)I_top, (const T *)I_rays,
                             (const T *)dL_dI, (const T *)dL_dJ, (T *)dL_dchi, (T *)dL_dS, (T *)dL_dIbottom,
                             (T *)dL_dItop, ray_group, checkpoint_levels);
    }
    return VRT_OK;
  });
}

vrt_status vrt_grid_solution_id(vrt_grid g, int64_t *id) {
  if (!g || !id) return VRT_E_ARG;
  *id = g->solution_id;
  return VRT_OK;
}

vrt_status vrt_formal_solution_vjp_last(vrt_grid g, vrt_prec prec, int32_t n_lambda, const void *chi, const void *S,
                                        const void *I_bottom, const void *I_top, const void *dL_dI,
                                        const void *dL_dJ, void *dL_dchi, void *dL_dS, void *dL_dIbottom,
                                        void *dL_dItop, int32_t ray_group, int64_t solution_id) {
  if (!g) return VRT_E_ARG;
  return guarded(g->ctx, [&] {
    if (!valid_prec(prec) || n_lambda <= 0 || ray_group < 0)
      fail(VRT_E_ARG, "bad precision, n_lambda or ray group");
    if (g->kind != 0) fail(VRT_E_ARG, "the reverse sweep exists for Voronoi grids only");
    if (g->segment) fail(VRT_E_ARG, "the reverse sweep differentiates the linear segment only");
    if (g->R == 0) fail(VRT_E_STATE, "rays not set");
    if (!chi || !S) fail(VRT_E_ARG, "chi and S are required");
    if (!dL_dI && !dL_dJ) fail(VRT_E_ARG, "give dL_dI, dL_dJ or both");
    if (solution_id != g->solution_id || !g->last_I || !g->last_own)
      fail(VRT_E_STATE, "the grid's last formal solution is not solution %lld", (long long)solution_id);
    if (g->last_nl != n_lambda || g->last_ld != n_lambda)
      fail(VRT_E_STATE, "the last solution had %d wavelengths in rows of %d", g->last_nl, g->last_ld);
    if (g->n == 0) return VRT_OK;
    // the last solution's rows of every ray, in this precision, in the
    // reverse sweep's own scratch (NaN if its persistent sweep raised an error)
    const size_t el = prec == VRT_F32 ? 4 : 8;
    const int64_t count = (int64_t)g->R * g->n * n_lambda;
    g->d_vIch.release();
    g->d_vIfr.release();
    g->d_vI.alloc((size_t)count * el);
    const int32_t *err = g->last_abs ? g->d_epoch.as<int32_t>() + 1 : nullptr;
    hipStream_t s = g->ctx->stream;
    if (prec == VRT_F32) {
      using T = float;
      T *Ifw = g->d_vI.as<T>();
      vrt::launch_rows_convert<T>(s, g->last_I, g->last_prec == VRT_F32, g->last_abs, Ifw, count, err);
      const T *ib = I_bottom ? (const T *)I_bottom : (const T *)S;
      formal_solution_vjp<T>(g, n_lambda, (const T *)chi, (const T *)S, ib, (const T *)I_top, Ifw,
                             (const T *)dL_dI, (const T *)dL_dJ, (T *)dL_dchi, (T *)dL_dS, (T *)dL_dIbottom,
                             (T *)dL_dItop, ray_group, 0);
    } else {
      using T = double;
      T *Ifw = g->d_vI.as<T>();
      vrt::launch_rows_convert<T>(s, g->last_I, g->last_prec == VRT_F32, g->last_abs, Ifw, count, err);
      const T *ib = I_bottom ? (const T *)I_bottom : (const T *)S;
      formal_solution_vjp<T>(g, n_lambda, (const T *)chi, (const T *)S, ib, (const T *)I_top, Ifw,
                             (const T *)dL_dI, (const T *)dL_dJ, (T *)dL_dchi, (T *)dL_dS, (T *)dL_dIbottom,
                             (T *)dL_dItop, ray_group, 0);
    }
    return VRT_OK;
  });
}

vrt_status vrt_formal_solution_vjp_scratch(vrt_grid g, vrt_prec prec, int32_t n_lambda, int32_t keep_intensities,
                                           int32_t ray_group, int32_t checkpoint_levels, int64_t *bytes) {
  if (!g) return VRT_E_ARG;
  return guarded(g->ctx, [&] {
    if (!valid_prec(prec) || n_lambda <= 0 || ray_group < 0 || checkpoint_levels < 0 || !bytes)
      fail(VRT_E_ARG, "bad precision, n_lambda, ray group, checkpoint interval or output");
    if (g->kind != 0) fail(VRT_E_ARG, "the reverse sweep exists for Voronoi grids only");
    if (g->R == 0) fail(VRT_E_STATE, "rays not set");
    const int64_t n = g->n, nl = n_lambda;
    const int64_t el = prec == VRT_F32 ? 4 : 8;
    const int32_t group = ray_group <= 0 || ray_group > g->R ? g->R : ray_group;
    int64_t rows = 3 * (int64_t)group * n;  // adjoint, S and chi contributions of a ray group
    int64_t extra = 4 * n * nl * 8;         // double accumulators
    if (!keep_intensities) {
      if (checkpoint_levels > 0 && n > 0) {
        build_checkpoints(g, std::min(checkpoint_levels, std::max(g->n_steps, 1)), group);
        rows += std::max<int64_t>(g->ck_chunk_rows, 1) + std::max<int64_t>(g->ck_front_rows, 1);
        extra += g->n_rec * (int64_t)sizeof(int4);
      } else {
        rows += (int64_t)group * n;
      }
    }
    *bytes = rows * nl * el + extra;
    return VRT_OK;
  });
}

vrt_status vrt_emergent_scatter(vrt_grid g, vrt_prec prec, int32_t n_lambda, const void *dL_dIem, void *dL_dI) {
  if (!g) return VRT_E_ARG;
  return guarded(g->ctx, [&] {
    if (!valid_prec(prec) || n_lambda <= 0) fail(VRT_E_ARG, "bad precision or n_lambda");
    if (g->R == 0) fail(VRT_E_STATE, "rays not set");
    const int64_t total = g->em_off.back();
    const int64_t full = (int64_t)g->R * g->n * n_lambda;
    if (full > 0 && !dL_dI) fail(VRT_E_ARG, "null output");
    if (total > 0 && !dL_dIem) fail(VRT_E_ARG, "null input");
    hipStream_t s = g->ctx->stream;
    if (prec == VRT_F32) {
      vrt::launch_fill_zero<float>(s, full, (float *)dL_dI);
      vrt::launch_emergent_scatter<float>(s, total, n_lambda, g->n, g->d_em_ray.as<int32_t>(),
                                          g->d_em_site.as<int32_t>(), (const float *)dL_dIem, (float *)dL_dI);
    } else {
      vrt::launch_fill_zero<double>(s, full, (double *)dL_dI);
      vrt::launch_emergent_scatter<double>(s, total, n_lambda, g->n, g->d_em_ray.as<int32_t>(),
                                           g->d_em_site.as<int32_t>(), (const double *)dL_dIem, (double *)dL_dI);
    }
    return VRT_OK;
  });
}

vrt_status vrt_lte_continuum_vjp(vrt_grid g, vrt_prec prec, int32_t n_lambda, const double *lambda_m, double kappa0,
                                 const double *T, const double *rho, const void *dL_dchi, const void *dL_dS,
                                 const void *dL_dIbottom, double *dL_dT, double *dL_drho) {
  if (!g) return VRT_E_ARG;
  return guarded(g->ctx, [&] {
    if (!valid_prec(prec) || n_lambda <= 0 || !lambda_m) fail(VRT_E_ARG, "bad LTE adjoint arguments");
    if (g->n == 0) return VRT_OK;
    if (!T || !rho || !dL_dchi || !dL_dS || !dL_dT || !dL_drho) fail(VRT_E_ARG, "null device array");
    hipStream_t s = g->ctx->stream;
    if (g->h_lam.size() != (size_t)n_lambda || !std::equal(g->h_lam.begin(), g->h_lam.end(), lambda_m)) {
      VRT_HIP(hipStreamSynchronize(s));
      g->d_lam.alloc((size_t)n_lambda * sizeof(double));
      VRT_HIP(hipMemcpy(g->d_lam.p, lambda_m, (size_t)n_lambda * sizeof(double), hipMemcpyHostToDevice));
      g->h_lam.assign(lambda_m, lambda_m + n_lambda);
    }
    if (prec == VRT_F32)
      vrt::launch_lte_vjp<float>(s, g->n, n_lambda, g->d_lam.as<double>(), kappa0, T, rho, (const float *)dL_dchi,
                                 (const float *)dL_dS, (const float *)dL_dIbottom, dL_dT, dL_drho);
    else
      vrt::launch_lte_vjp<double>(s, g->n, n_lambda, g->d_lam.as<double>(), kappa0, T, rho, (const double *)dL_dchi,
                                  (const double *)dL_dS, (const double *)dL_dIbottom, dL_dT, dL_drho);
    return VRT_OK;
  });
}

vrt_status vrt_grid_device_status(vrt_grid g) {
  if (!g) return VRT_E_ARG;
  return guarded(g->ctx, [&] {
    VRT_HIP(hipStreamSynchronize(g->ctx->stream));
    take_device_error(g, 0);
    return VRT_OK;
  });
}

vrt_status vrt_grid_emergent_index(vrt_grid g, int64_t *offsets, int32_t *sites) {
  if (!g) return VRT_E_ARG;
  if (g->R == 0) {
    g->ctx->err = "rays not set";
    return VRT_E_STATE;
  }
  if (offsets) std::copy(g->em_off.begin(), g->em_off.end(), offsets);
  if (sites) std::copy(g->em_site.begin(), g->em_site.end(), sites);
  return VRT_OK;
}

vrt_status vrt_emergent_gather(vrt_grid g, vrt_prec prec, int32_t n_lambda, const void *I_rays, void *out) {
  if (!g) return VRT_E_ARG;
  return guarded(g->ctx, [&] {
    if (!valid_prec(prec) || n_lambda <= 0) fail(VRT_E_ARG, "bad precision or n_lambda");
    if (g->R == 0) fail(VRT_E_STATE, "rays not set");
    const void *I = I_rays ? I_rays : g->last_I;
    if (!I) fail(VRT_E_STATE, "no formal solution has run");
    int32_t ld = n_lambda;
    const bool ab = !I_rays && g->last_abs;
    if (!I_rays) {
      if (prec != g->last_prec || n_lambda != g->last_nl)
        fail(VRT_E_ARG, "the last solution had %d wavelengths in %s precision", g->last_nl,
             g->last_prec == VRT_F32 ? "single" : "double");
      ld = g->last_ld;
    }
    const int64_t total = g->em_off.back();
    if (total > 0 && !out) fail(VRT_E_ARG, "null output");
    const int32_t *err = ab ? g->d_epoch.as<int32_t>() + 1 : nullptr;
    if (prec == VRT_F32)
      vrt::launch_emergent<float>(g->ctx->stream, total, n_lambda, ld, g->n, g->d_em_ray.as<int32_t>(),
                                  g->d_em_site.as<int32_t>(), static_cast<const float *>(I), static_cast<float *>(out),
                                  ab, err);
    else
      vrt::launch_emergent<double>(g->ctx->stream, total, n_lambda, ld, g->n, g->d_em_ray.as<int32_t>(),
                                   g->d_em_site.as<int32_t>(), static_cast<const double *>(I),
                                   static_cast<double *>(out), ab, err);
    return VRT_OK;
  });
}

vrt_status vrt_idw_map(vrt_grid vor, vrt_grid reg, double power, int32_t *idx, double *w1, double *d2) {
  if (!vor || !reg) return VRT_E_ARG;
  return guarded(reg->ctx, [&] {
    if (vor->ctx != reg->ctx) fail(VRT_E_ARG, "the two grids belong to different contexts");
    if (vor->kind != 0 || reg->kind != 1) fail(VRT_E_ARG, "expected a Voronoi grid and a regular grid");
    if (vor->n < 1) fail(VRT_E_ARG, "the Voronoi grid has no sites");
    if (!(power > 0.0) || !std::isfinite(power)) fail(VRT_E_ARG, "power must be positive and finite");
    if (!idx || !w1) fail(VRT_E_ARG, "null output");
    const double Lx = vor->hi[0] - vor->lo[0], Ly = vor->hi[1] - vor->lo[1];
    const double X = (double)(reg->nx - 1) * reg->dx, Y = (double)(reg->ny - 1) * reg->dy;
    if (vor->periodic) {
      // one period in both grids, and boxes close enough that a difference of
      // coordinates needs at most one period shift
      if (std::fabs((double)reg->nx * reg->dx - Lx) > 1e-9 * Lx || std::fabs((double)reg->ny * reg->dy - Ly) > 1e-9 * Ly)
        fail(VRT_E_ARG, "the regular grid's periods (%g, %g) differ from the Voronoi box (%g, %g)",
             (double)reg->nx * reg->dx, (double)reg->ny * reg->dy, Lx, Ly);
      if (std::fabs(vor->lo[0]) > 0.5 * Lx || std::fabs(vor->lo[1]) > 0.5 * Ly)
        fail(VRT_E_ARG, "the Voronoi box must start within half a period of x = y = 0");
    } else if (vor->lo[0] > 0.0 || vor->lo[1] > 0.0 || X > vor->hi[0] || Y > vor->hi[1]) {
      fail(VRT_E_ARG, "regular points outside the Voronoi box in x or y");
    }
    if (reg->h_z.front() < vor->lo[2] || reg->h_z.back() > vor->hi[2])
      fail(VRT_E_ARG, "regular planes outside the Voronoi box in z");
    hipStream_t s = reg->ctx->stream;
    reg->d_walk_bad.alloc(sizeof(unsigned long long));
    vrt::launch_zero_u64(s, 1, reg->d_walk_bad.as<unsigned long long>());
    int32_t *bad = reg->d_walk_bad.as<int32_t>();
    // brute force on the finest lattice whose work (points x sites) stays
    // under 2^24 distances, then halve the stride
    auto lattice_points = [&](int64_t st) {
      return ((reg->nx + st - 1) / st) * ((reg->ny + st - 1) / st) * ((reg->nz + st - 1) / st);
    };
    int32_t s0 = 1;
    while (lattice_points(s0) > 1 && lattice_points(s0) * vor->n > (int64_t(1) << 24)) s0 *= 2;
    const int64_t pairs = vrt::idw_brute_scratch_pairs(reg->nx, reg->ny, reg->nz, s0, vor->n);
    reg->d_brute.alloc((size_t)pairs * 2 * (sizeof(int32_t) + sizeof(double)));
    double *pe = reg->d_brute.as<double>();
    int32_t *pb = reinterpret_cast<int32_t *>(pe + 2 * pairs);
    vrt::launch_idw_brute(s, reg->nx, reg->ny, reg->nz, reg->dx, reg->dy, reg->d_z.as<double>(), s0, vor->n,
                          vor->d_xyz.as<double>(), vor->periodic, Lx, Ly, power, idx, w1, d2, pb, pe);
    for (int32_t st = s0 / 2; st >= 1; st /= 2)
      vrt::launch_idw_level(s, reg->nx, reg->ny, reg->nz, reg->dx, reg->dy, reg->d_z.as<double>(), st, 2 * st,
                            vor->n, vor->d_xyz.as<double>(), vor->d_ptr.as<int64_t>(), vor->d_idx.as<int32_t>(),
                            vor->periodic, Lx, Ly, power, idx, w1, d2, bad);
    int32_t h_bad = 0;
    VRT_HIP(hipMemcpyAsync(&h_bad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    VRT_HIP(hipStreamSynchronize(s));
    if (h_bad) fail(VRT_E_GRID, "the nearest-site walk did not settle: the neighbour lists are incomplete");
    return VRT_OK;
  });
}

vrt_status vrt_idw_apply(vrt_grid vor, vrt_grid reg, int32_t n_cols, const int32_t *idx, const double *w1,
                         const double *src, double *dst) {
  if (!vor || !reg) return VRT_E_ARG;
  return guarded(reg->ctx, [&] {
    if (vor->ctx != reg->ctx) fail(VRT_E_ARG, "the two grids belong to different contexts");
    if (vor->kind != 0 || reg->kind != 1) fail(VRT_E_ARG, "expected a Voronoi grid and a regular grid");
    if (n_cols <= 0 || !idx || !w1 || !src || !dst) fail(VRT_E_ARG, "bad interpolation arguments");
    vrt::launch_idw_apply(reg->ctx->stream, reg->n, n_cols, vor->n, idx, w1, src, dst);
    return VRT_OK;
  });
}

vrt_status vrt_synthesis_vertical(vrt_grid vor, vrt_grid reg, vrt_prec prec, int32_t n_lambda, const int32_t *idx,
                                  const double *w1, const double *S_line, const void *phi, const double *chi_line,
                                  const double *chi_cont, const double *B, const void *I_bottom, void *I_top) {
  if (!vor || !reg) return VRT_E_ARG;
  return guarded(reg->ctx, [&] {
    if (vor->ctx != reg->ctx) fail(VRT_E_ARG, "the two grids belong to different contexts");
    if (vor->kind != 0 || reg->kind != 1) fail(VRT_E_ARG, "expected a Voronoi grid and a regular grid");
    if (!valid_prec(prec) || n_lambda <= 0) fail(VRT_E_ARG, "bad precision or n_lambda");
    if (!idx || !w1 || !S_line || !phi || !chi_line || !chi_cont || !B || !I_top)
      fail(VRT_E_ARG, "null argument");
    hipStream_t s = reg->ctx->stream;
    const int64_t m = reg->n, ncol = (int64_t)reg->nx * reg->ny;
    const double *z = reg->d_z.as<double>();
    reg->d_pack.alloc((size_t)m * 4 * (prec == VRT_F32 ? sizeof(float) : sizeof(double)));
    if (prec == VRT_F32) {
      vrt::launch_line_pack<float>(s, m, vor->n, idx, w1, S_line, chi_line, chi_cont, B, reg->d_pack.p);
      vrt::launch_vertical_line<float>(s, ncol, reg->nz, n_lambda, z, static_cast<const float *>(phi), reg->d_pack.p,
                                       B, static_cast<const float *>(I_bottom), static_cast<float *>(I_top));
    } else {
      vrt::launch_line_pack<double>(s, m, vor->n, idx, w1, S_line, chi_line, chi_cont, B, reg->d_pack.p);
      vrt::launch_vertical_line<double>(s, ncol, reg->nz, n_lambda, z, static_cast<const double *>(phi),
                                        reg->d_pack.p, B, static_cast<const double *>(I_bottom),
                                        static_cast<double *>(I_top));
    }
    return VRT_OK;
  });
}

vrt_status vrt_lc_vertical(vrt_grid reg, vrt_prec prec, int32_t n_lambda, const void *chi, const void *S,
                           const void *I_bottom, void *I_top) {
  if (!reg) return VRT_E_ARG;
  return guarded(reg->ctx, [&] {
    if (reg->kind != 1) fail(VRT_E_ARG, "expected a regular grid");
    if (!valid_prec(prec) || n_lambda <= 0 || !chi || !S || !I_top) fail(VRT_E_ARG, "bad arguments");
    hipStream_t s = reg->ctx->stream;
    const int64_t ncol = (int64_t)reg->nx * reg->ny;
    const double *z = reg->d_z.as<double>();
    if (prec == VRT_F32)
      vrt::launch_vertical_plain<float>(s, ncol, reg->nz, n_lambda, z, static_cast<const float *>(chi),
                                        static_cast<const float *>(S), static_cast<const float *>(I_bottom),
                                        static_cast<float *>(I_top));
    else
      vrt::launch_vertical_plain<double>(s, ncol, reg->nz, n_lambda, z, static_cast<const double *>(chi),
                                         static_cast<const double *>(S), static_cast<const double *>(I_bottom),
                                         static_cast<double *>(I_top));
    return VRT_OK;
  });
}

}  // extern "C"
