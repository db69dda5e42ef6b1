// Persistent, dataflow-ordered Voronoi sweep: the whole formal solution of
// every ray in one launch instead of one launch per level step.
//
// Work is the step-major sweep record list (level step 0 of every ray, then
// step 1, ...), cut into wave items of at most 64/C records of one (level
// step, ray) segment (records of one step are independent of each other, so
// no item waits on itself). The item table carries the ray, so the buffer
// descriptor of the ray's intensity rows is uniform across the wavefront.
//
// Ranks. Every wavefront first registers in a counter; the first one to
// register waits until the whole grid has registered, or until the count has
// stopped growing for a while, then freezes the counter and publishes the
// count W. A wavefront that registered before the freeze has a rank q < W
// and walks items q, q + W, q + 2W, ... in increasing order; one that
// registers after the freeze (a workgroup that was not resident) does
// nothing. Only running wavefronts therefore hold work. The occupancy the
// runtime reports cannot promise that by itself: it counts vector registers,
// and a kernel with more than about 80 scalar registers fits one wavefront
// per SIMD fewer than reported (measured: with 86 to 98 scalar registers a
// grid sized that way was never wholly resident, with 71 it was). The
// kernels are compiled with at most 80 scalar registers, so the whole grid
// is normally resident and the freeze comes as soon as the last wavefront
// has registered.
//
// Dataflow. Before updating a site a lane waits until both of its upwind
// sites carry the current epoch stamp in a per-(ray, site) flag; after
// writing the site's intensity row the wave stamps the site. Upwind sites
// always sit in earlier items, and the wavefront that owns the earliest
// unfinished item has finished all its own earlier items, so that item can
// always proceed: the sweep cannot deadlock. Each wait is bounded anyway; a
// wave that exceeds the bound raises a device error flag, every other waiting
// wave then stops waiting, and the launch drains.
//
// Coherence without cache maintenance. The eight dies have separate L2
// caches, and the agent-scope fences that order plain accesses write back
// and invalidate a whole L2 at every handshake (a sweep built on them took
// 49 ms). Instead every access to the data that passes between wavefronts
// carries the device-scope cache policy (sc1): the intensity rows are stored
// and loaded through buffer descriptors with sc1, and the stamps, polls and
// registration words are relaxed agent-scope atomics. A wave waits for its
// row stores to complete (vmcnt 0) before it stamps, and reads an upwind row
// only after it has seen the row's stamp. chi, S and the boundary rows are
// only read, so they stay cached.
//
// Flags hold an epoch number that a one-thread kernel increments before each
// sweep (and the registration words are cleared there), so the flags never
// need clearing between sweeps.

#include "persist.h"
#include "segment.h"
#include "vrt_internal.h"

namespace {

template <typename T, int V> struct PLane {
  typedef T type __attribute__((ext_vector_type(V)));
  static __device__ __forceinline__ type load(const T *p) { return *reinterpret_cast<const type *>(p); }
  static __device__ __forceinline__ T get(const type &v, int k) { return v[k]; }
  static __device__ __forceinline__ void set(type &v, int k, T x) { v[k] = x; }
};
template <typename T> struct PLane<T, 1> {
  typedef T type;
  static __device__ __forceinline__ type load(const T *p) { return *p; }
  static __device__ __forceinline__ T get(const type &v, int) { return v; }
  static __device__ __forceinline__ void set(type &v, int, T x) { v = x; }
};

using namespace vrt_persist;

// words: [0] epoch of the stamped sweeps, [1] device error (bit 0 a wait gave
// up, bit 1 a negative or NaN intensity in a sign-encoded sweep), [2]
// registration word (count, plus kFrozen once frozen), [3] frozen count + 1 (0
// until frozen), [5] epoch of the sign-encoded sweeps
__global__ void begin_kernel(int32_t *words, int32_t which) {
  words[which] += 1;
  words[2] = 0;
  words[3] = 0;
}

// Sign-encoded rows: the intensities of the linear-segment sweep are never
// negative (S >= 0, non-negative segment weights and boundary values), so a
// sweep of odd epoch stores -I and one of even epoch +I, and a consumer knows
// an upwind row is this sweep's once every element it loaded carries the
// epoch's sign. The previous sweep's rows carry the other sign, so no stamps,
// no per-sweep reset and no store-to-stamp ordering are needed. Rows are read
// back as |I|.
template <typename T> __device__ __forceinline__ T abs_el(T x) {
  if constexpr (sizeof(T) == 4) return __builtin_fabsf(x);
  else return __builtin_fabs(x);
}

// fills a sign-encoded block with zeros of the current epoch's sign, so that
// the next epoch reads none of it as written
template <typename T> __global__ void sign_fill_kernel(T *__restrict__ p, int64_t count, const int32_t *words) {
  const T z = (words[5] & 1) ? -T(0) : T(0);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
    p[t] = z;
}

// item_rec[i] = first record of wave item i, item_cnt[i] = its record count
// (<= 64/C) + 256 x its ray
// Row access of the persistent sweep. Stamped: plain device-scope load and
// store. Sign-encoded: the load is repeated (bounded, like a stamp wait) until
// every element carries the epoch's sign and is returned as |I|; the store
// writes the epoch's sign and flags a negative or NaN value, which the encoding
// cannot carry.
template <typename T, typename VT, typename L, int V, bool SIGN, bool BIG>
__device__ __forceinline__ VT get_row(const RayBlock<BIG> &r, int64_t off, bool neg, int32_t *err, int64_t cap) {
  VT u = r.template load<VT>(off);
  if constexpr (SIGN) {
    auto ready = [&](const VT &x) {
      bool ok = true;
#pragma unroll
      for (int k = 0; k < V; ++k) ok = ok && ((__builtin_signbit(L::get(x, k)) != 0) == neg);
      return ok;
    };
    int64_t it = 0;
    while (!ready(u)) {
      ++it;
      if ((it & 63) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, kXScope) != 0) break;
      if (it > cap) {
        __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, kXScope);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      u = r.template load<VT>(off);
    }
#pragma unroll
    for (int k = 0; k < V; ++k) L::set(u, k, abs_el<T>(L::get(u, k)));
  }
  return u;
}

template <typename T, typename VT, typename L, int V, bool SIGN, bool BIG>
__device__ __forceinline__ void put_row(const RayBlock<BIG> &r, int64_t off, VT v, bool neg, int32_t *err) {
  if constexpr (SIGN) {
    bool bad = false;
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const T x = L::get(v, k);
      bad = bad || !(x >= T(0));
      const T a = abs_el<T>(x);
      L::set(v, k, neg ? -a : a);
    }
    if (bad) __hip_atomic_fetch_or(err, 2, __ATOMIC_RELAXED, kXScope);
  }
  r.template store<VT>(off, v);
}

template <typename T, int C, int V, bool SIGN, bool BIG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_num_sgpr(80))) void persistent_sweep_kernel(
    const int4 *__restrict__ ri, const typename vrt::RecOf<T>::type *__restrict__ rf,
    const int64_t *__restrict__ item_rec, const int32_t *__restrict__ item_cnt, int64_t n_items, int32_t nl,
    int64_t cs, int64_t n, int64_t flag_ld, const T *__restrict__ chi, const T *__restrict__ S,
    const T *__restrict__ Ibot, const T *__restrict__ Itop, T *I, int32_t *flags, int32_t *words, int64_t spin_cap,
    int64_t mixed_bytes) {
  using L = PLane<T, V>;
  using VT = typename L::type;
  const int32_t epoch = SIGN ? words[5] : words[0];
  // mixed_bytes > 0: items mix rays (records of one level step in site order
  // across rays); the row block then covers every ray's rows (mixed_bytes of
  // them; BIG when that is 4 GiB or more) and each lane adds its own ray's
  // offset
  const bool mixed = mixed_bytes > 0;
  int32_t *err = words + 1;
  // a sign-encoded sweep after an unacknowledged error would trust rows of an
  // unknown sign: it does nothing until the host has read and cleared the error
  if (SIGN && __hip_atomic_load(err, __ATOMIC_RELAXED, kXScope) != 0) return;
  const bool neg = (epoch & 1) != 0;
  const int lane = threadIdx.x & 63;
  int64_t W = 0;
  const int64_t rank = register_wave(words, (int32_t)(gridDim.x * (blockDim.x >> 6)), spin_cap, lane, W);
  if (rank < 0) return;
  const int l0 = (lane % C) * V;
  const int sub = lane / C;
  for (int64_t item = rank; item < n_items; item += W) {
    const int32_t cr = item_cnt[item];
    const bool live = sub < (cr & 255);
    const int64_t rec = item_rec[item] + sub;
    int4 q = make_int4(0, -1, -1, 0);
    if (live) q = ri[rec];
    const int32_t site = q.x, k1 = q.y, k2 = q.z, ray = q.w >> 1;
    const bool up = (q.w & 1) != 0;
    int32_t *fr = flags + (int64_t)ray * flag_ld;
    if (!SIGN && live && k1 >= 0) {
      if (wait_stamp(fr + k1, epoch, err, spin_cap) && k2 >= 0) wait_stamp(fr + k2, epoch, err, spin_cap);
    }
    if (live) {
      // the item's ray's block of n * nl values (BIG: 4 GiB or more), or every
      // ray's rows for mixed items
      const RayBlock<BIG> Iray(mixed ? I : I + (int64_t)(cr >> 8) * n * nl,
                               mixed ? mixed_bytes : n * nl * (int64_t)sizeof(T));
      const int64_t rb = mixed ? (int64_t)ray * n * nl : 0;
      // input rows (chi, S, boundary intensities) of site i at i cs (cs >= nl)
      const int64_t bi = (int64_t)site * nl, ei = (int64_t)site * cs;
      if (k1 < 0) {
        for (int l = l0; l < nl; l += C * V) {
          VT v;
          if (up) v = L::load(Ibot + ei + l);
          else if (Itop) v = L::load(Itop + ei + l);
          else v = VT(T(0));
          put_row<T, VT, L, V, SIGN>(Iray, (rb + bi + l) * (int64_t)sizeof(T), v, neg, err);
        }
      } else {
        const auto f = rf[rec];
        const T w1 = f.w1, w2 = T(1) - f.w1;
        const T h1 = T(0.5) * f.ds1, h2 = T(0.5) * f.ds2;
        const bool two = k2 >= 0;
        const int64_t b1 = (int64_t)k1 * nl;
        const int64_t b2 = (int64_t)(two ? k2 : k1) * nl;
        const int64_t e1 = (int64_t)k1 * cs, e2 = (int64_t)(two ? k2 : k1) * cs;
        for (int l = l0; l < nl; l += C * V) {
          const VT ci = L::load(chi + ei + l), si = L::load(S + ei + l);
          const VT c1 = L::load(chi + e1 + l), s1 = L::load(S + e1 + l);
          const VT u1 = get_row<T, VT, L, V, SIGN>(Iray, (rb + b1 + l) * (int64_t)sizeof(T), neg, err, spin_cap);
          VT c2, s2, u2;
          if (two) {
            c2 = L::load(chi + e2 + l);
            s2 = L::load(S + e2 + l);
            u2 = get_row<T, VT, L, V, SIGN>(Iray, (rb + b2 + l) * (int64_t)sizeof(T), neg, err, spin_cap);
          }
          VT out;
#pragma unroll
          for (int k = 0; k < V; ++k) {
            const T cik = L::get(ci, k), sik = L::get(si, k);
            T Iv = vrt::seg_line<T>((L::get(c1, k) + cik) * h1, L::get(u1, k), L::get(s1, k), sik);
            if (two) {
              const T Ib = vrt::seg_line<T>((L::get(c2, k) + cik) * h2, L::get(u2, k), L::get(s2, k), sik);
              Iv = vrt::seg_mix<T>(w1, w2, Iv, Ib);
            }
            L::set(out, k, Iv);
          }
          put_row<T, VT, L, V, SIGN>(Iray, (rb + bi + l) * (int64_t)sizeof(T), out, neg, err);
        }
      }
    }
    if constexpr (!SIGN) {
      // every row store of the wave has completed before any of its stamps
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      __builtin_amdgcn_s_waitcnt(0);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (live && (lane % C) == 0) __hip_atomic_store(fr + site, epoch, __ATOMIC_RELAXED, kXScope);
    }
  }
}

template <typename T, int C, int V>
void launch_pc(hipStream_t s, const vrt::PersistItems &it, int32_t max_blocks, const int4 *ri,
               const typename vrt::RecOf<T>::type *rf, int32_t nl, int64_t cs, int64_t n, int64_t flag_ld,
               const T *chi, const T *S, const T *Ibot, const T *Itop, T *I, int32_t *flags, int32_t *words,
               int64_t cap, bool sign, int64_t mixed_bytes) {
  if (it.spw != 64 / C) throw vrt::Error(VRT_E_STATE, "persistent item table built for another record width");
  const int64_t block = mixed_bytes > 0 ? mixed_bytes : n * (int64_t)nl * (int64_t)sizeof(T);
  const bool big = block >= (int64_t(1) << 32);
  auto kern = sign ? (big ? persistent_sweep_kernel<T, C, V, true, true> : persistent_sweep_kernel<T, C, V, true, false>)
                   : (big ? persistent_sweep_kernel<T, C, V, false, true> : persistent_sweep_kernel<T, C, V, false, false>);
  int dev = 0, cus = 0, per_cu = 0;
  VRT_HIP(hipGetDevice(&dev));
  VRT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  VRT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0));
  if (per_cu < 1) throw vrt::Error(VRT_E_HIP, "persistent sweep kernel cannot be resident");
  // as many workgroups as the runtime says can be resident, at most one wave
  // item per wavefront, unless the caller set the count (registration gives
  // work only to those that run, so any count is correct)
  int64_t blocks = (int64_t)cus * per_cu;
  if (blocks > (it.n_items + 3) / 4) blocks = (it.n_items + 3) / 4;
  if (max_blocks > 0) blocks = max_blocks;
  if (blocks < 1) blocks = 1;
  const int64_t *item_rec = it.rec.as<int64_t>();
  const int32_t *item_cnt = it.cnt.as<int32_t>();
  const int64_t n_items = it.n_items;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, s, ri, rf, item_rec, item_cnt, n_items, nl, cs, n,
                     flag_ld, chi, S, Ibot, Itop, I, flags, words, cap, mixed_bytes);
  VRT_HIP(hipGetLastError());
}

template <typename T, int V>
void launch_pv(hipStream_t s, const vrt::PersistItems &it, int32_t mb, const int4 *ri,
               const typename vrt::RecOf<T>::type *rf, int32_t nl, int64_t cs, int64_t n, int64_t fl, const T *chi,
               const T *S, const T *Ibot, const T *Itop, T *I, int32_t *flags, int32_t *words, int64_t cap, bool sg,
               int64_t mx) {
  switch (vrt::lanes_per_record(nl / V)) {
    case 64: launch_pc<T, 64, V>(s, it, mb, ri, rf, nl, cs, n, fl, chi, S, Ibot, Itop, I, flags, words, cap, sg, mx); break;
    case 32: launch_pc<T, 32, V>(s, it, mb, ri, rf, nl, cs, n, fl, chi, S, Ibot, Itop, I, flags, words, cap, sg, mx); break;
    case 16: launch_pc<T, 16, V>(s, it, mb, ri, rf, nl, cs, n, fl, chi, S, Ibot, Itop, I, flags, words, cap, sg, mx); break;
    case 8: launch_pc<T, 8, V>(s, it, mb, ri, rf, nl, cs, n, fl, chi, S, Ibot, Itop, I, flags, words, cap, sg, mx); break;
    case 4: launch_pc<T, 4, V>(s, it, mb, ri, rf, nl, cs, n, fl, chi, S, Ibot, Itop, I, flags, words, cap, sg, mx); break;
    case 2: launch_pc<T, 2, V>(s, it, mb, ri, rf, nl, cs, n, fl, chi, S, Ibot, Itop, I, flags, words, cap, sg, mx); break;
    default: launch_pc<T, 1, V>(s, it, mb, ri, rf, nl, cs, n, fl, chi, S, Ibot, Itop, I, flags, words, cap, sg, mx); break;
  }
}

}  // namespace

namespace vrt {

bool al16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

void launch_persist_begin(hipStream_t s, int32_t *words, bool sign) {
  hipLaunchKernelGGL(begin_kernel, dim3(1), dim3(1), 0, s, words, sign ? 5 : 0);
  VRT_HIP(hipGetLastError());
}

template <typename T> void launch_sign_fill(hipStream_t s, T *p, int64_t count, const int32_t *words) {
  if (count <= 0) return;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(sign_fill_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, count, words);
  VRT_HIP(hipGetLastError());
}
template void launch_sign_fill<float>(hipStream_t, float *, int64_t, const int32_t *);
template void launch_sign_fill<double>(hipStream_t, double *, int64_t, const int32_t *);

int32_t persistent_records_per_wave(int32_t nl, int elem_bytes, bool aligned, int64_t cs) {
  const int VW = 16 / elem_bytes;
  const int V = (aligned && nl % VW == 0 && cs % VW == 0) ? VW : 1;
  return 64 / lanes_per_record(nl / V);
}

template <typename T>
void launch_persistent_sweep(hipStream_t s, const PersistItems &items, int32_t max_blocks, const int4 *ri,
                             const typename RecOf<T>::type *rf, int32_t nl, int64_t cs, int64_t n, int64_t flag_ld,
                             const T *chi, const T *S, const T *Ibot, const T *Itop, T *I, int32_t *flags,
                             int32_t *words, int64_t spin_cap, bool sign, int32_t mixed_rays) {
  if (items.n_items <= 0) return;
  const int64_t mixed_bytes = mixed_rays > 0 ? (int64_t)mixed_rays * n * (int64_t)nl * (int64_t)sizeof(T) : 0;
  constexpr int VW = 16 / sizeof(T);
  const bool aligned = al16(chi) && al16(S) && al16(Ibot) && al16(Itop) && al16(I);
  if (aligned && nl % VW == 0 && cs % VW == 0)
    launch_pv<T, VW>(s, items, max_blocks, ri, rf, nl, cs, n, flag_ld, chi, S, Ibot, Itop, I, flags, words, spin_cap,
                     sign, mixed_bytes);
  else
    launch_pv<T, 1>(s, items, max_blocks, ri, rf, nl, cs, n, flag_ld, chi, S, Ibot, Itop, I, flags, words, spin_cap,
                    sign, mixed_bytes);
}

template void launch_persistent_sweep<float>(hipStream_t, const PersistItems &, int32_t, const int4 *, const RecF32 *,
                                             int32_t, int64_t, int64_t, int64_t, const float *, const float *,
                                             const float *, const float *, float *, int32_t *, int32_t *, int64_t,
                                             bool, int32_t);
template void launch_persistent_sweep<double>(hipStream_t, const PersistItems &, int32_t, const int4 *,
                                              const RecF64 *, int32_t, int64_t, int64_t, int64_t, const double *,
                                              const double *, const double *, const double *, double *, int32_t *,
                                              int32_t *, int64_t, bool, int32_t);

}  // namespace vrt
