// Persistent, dataflow-ordered Voronoi sweep: the whole formal solution of
// every ray in one cooperative launch instead of one launch per level.
//
// Work is the step-major sweep record list (level 0 of every ray, then level
// 1, ...), cut into wave items of at most 64/C records that never straddle a
// level step (records of one step are independent of each other, so no item
// waits on itself). Every wavefront of the grid is
// resident (cooperative launch) and walks the items w, w + W, w + 2W, ... in
// increasing order (W = number of wavefronts). Before updating a site it waits
// until both of its upwind sites carry the current epoch stamp in a
// per-(ray, site) flag; after writing the site's intensity row it publishes
// the row (release at agent scope) and stamps the site's flag. Upwind sites
// always sit in earlier items, and the wave that owns the earliest unfinished
// item has finished all its own earlier items, so that item can always
// proceed: the sweep cannot deadlock. Each wait is bounded anyway; a wave that
// exceeds the bound raises a device error flag, every other waiting wave sees
// it and stops waiting, and the launch always drains.
//
// Flags hold an epoch number that a one-thread kernel increments before each
// sweep, so they never need clearing between sweeps.

#include "segment.h"
#include "vrt_internal.h"

namespace {

template <typename T, int V> struct PLane {
  typedef T type __attribute__((ext_vector_type(V)));
  static __device__ __forceinline__ type load(const T *p) { return *reinterpret_cast<const type *>(p); }
  static __device__ __forceinline__ void store(T *p, const type &v) { *reinterpret_cast<type *>(p) = v; }
  static __device__ __forceinline__ T get(const type &v, int k) { return v[k]; }
  static __device__ __forceinline__ void set(type &v, int k, T x) { v[k] = x; }
};
template <typename T> struct PLane<T, 1> {
  typedef T type;
  static __device__ __forceinline__ type load(const T *p) { return *p; }
  static __device__ __forceinline__ void store(T *p, const type &v) { *p = v; }
  static __device__ __forceinline__ T get(const type &v, int) { return v; }
  static __device__ __forceinline__ void set(type &v, int, T x) { v = x; }
};

__global__ void epoch_kernel(int32_t *epoch) { *epoch += 1; }

// Wait until *f == epoch. Returns false if the bound was exceeded or another
// wave already gave up (then the caller proceeds without the data).
__device__ __forceinline__ bool wait_stamp(const int32_t *f, int32_t epoch, int32_t *err, int64_t cap) {
  int64_t it = 0;
  while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
    ++it;
    if ((it & 63) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if (it > cap) {
      __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

// item_rec[i] = first record of wave item i, item_cnt[i] = its record count (<= 64/C)
template <typename T, int C, int V>
__global__ __launch_bounds__(256) void persistent_sweep_kernel(
    const int4 *__restrict__ ri, const typename vrt::RecOf<T>::type *__restrict__ rf,
    const int64_t *__restrict__ item_rec, const int32_t *__restrict__ item_cnt, int64_t n_items, int32_t nl,
    int64_t n, const T *__restrict__ chi, const T *__restrict__ S, const T *__restrict__ Ibot,
    const T *__restrict__ Itop, T *I, int32_t *flags, const int32_t *__restrict__ epoch_p, int32_t *err,
    int64_t spin_cap) {
  using L = PLane<T, V>;
  using VT = typename L::type;
  const int32_t epoch = *epoch_p;
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t W = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int l0 = (lane % C) * V;
  for (int64_t item = gw; item < n_items; item += W) {
    const int sub = lane / C;
    const bool live = sub < item_cnt[item];
    const int64_t rec = item_rec[item] + sub;
    int4 q = make_int4(0, -1, -1, 0);
    if (live) q = ri[rec];
    const int32_t site = q.x, k1 = q.y, k2 = q.z, ray = q.w >> 1;
    const bool up = (q.w & 1) != 0;
    int32_t *fr = flags + (int64_t)ray * n;
    if (live && k1 >= 0) {
      if (wait_stamp(fr + k1, epoch, err, spin_cap) && k2 >= 0) wait_stamp(fr + k2, epoch, err, spin_cap);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (live) {
      T *Iray = I + (int64_t)ray * n * nl;
      const int64_t bi = (int64_t)site * nl;
      if (k1 < 0) {
        for (int l = l0; l < nl; l += C * V) {
          VT v;
          if (up) v = L::load(Ibot + bi + l);
          else if (Itop) v = L::load(Itop + bi + l);
          else v = VT(T(0));
          L::store(Iray + bi + l, v);
        }
      } else {
        const auto f = rf[rec];
        const T w1 = f.w1, w2 = T(1) - f.w1;
        const T h1 = T(0.5) * f.ds1, h2 = T(0.5) * f.ds2;
        const bool two = k2 >= 0;
        const int64_t b1 = (int64_t)k1 * nl;
        const int64_t b2 = (int64_t)(two ? k2 : k1) * nl;
        for (int l = l0; l < nl; l += C * V) {
          const VT ci = L::load(chi + bi + l), si = L::load(S + bi + l);
          const VT c1 = L::load(chi + b1 + l), s1 = L::load(S + b1 + l), u1 = L::load(Iray + b1 + l);
          VT c2, s2, u2;
          if (two) {
            c2 = L::load(chi + b2 + l);
            s2 = L::load(S + b2 + l);
            u2 = L::load(Iray + b2 + l);
          }
          VT out;
#pragma unroll
          for (int k = 0; k < V; ++k) {
            const T cik = L::get(ci, k), sik = L::get(si, k);
            T E, pu, p0;
            vrt::Seg<T>::weights((L::get(c1, k) + cik) * h1, E, pu, p0);
            T Iv = E * L::get(u1, k) + pu * L::get(s1, k) + p0 * sik;
            if (two) {
              vrt::Seg<T>::weights((L::get(c2, k) + cik) * h2, E, pu, p0);
              const T Ib = E * L::get(u2, k) + pu * L::get(s2, k) + p0 * sik;
              Iv = w1 * Iv + w2 * Ib;
            }
            L::set(out, k, Iv);
          }
          L::store(Iray + bi + l, out);
        }
      }
    }
    // publish the rows written by every lane of the wave, then stamp the sites
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (live && (lane % C) == 0) __hip_atomic_store(fr + site, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename T, int C, int V>
void launch_pc(hipStream_t s, const vrt::PersistItems &it, int32_t max_blocks, const int4 *ri,
               const typename vrt::RecOf<T>::type *rf, int32_t nl, int64_t n, const T *chi, const T *S,
               const T *Ibot, const T *Itop, T *I, int32_t *flags, const int32_t *epoch, int32_t *err,
               int64_t cap) {
  if (it.spw != 64 / C) throw vrt::Error(VRT_E_STATE, "persistent item table built for another record width");
  auto kern = persistent_sweep_kernel<T, C, V>;
  int dev = 0, cus = 0, per_cu = 0;
  VRT_HIP(hipGetDevice(&dev));
  VRT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  VRT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0));
  if (per_cu < 1) throw vrt::Error(VRT_E_HIP, "persistent sweep kernel cannot be resident");
  const int64_t items = it.n_items;
  int64_t blocks = (int64_t)cus * per_cu;
  if (max_blocks > 0 && blocks > max_blocks) blocks = max_blocks;
  if (blocks > (items + 3) / 4) blocks = (items + 3) / 4;
  if (blocks < 1) blocks = 1;
  const int64_t *item_rec = it.rec.as<int64_t>();
  const int32_t *item_cnt = it.cnt.as<int32_t>();
  int64_t n_items = items;
  void *args[] = {(void *)&ri,  (void *)&rf,   (void *)&item_rec, (void *)&item_cnt, (void *)&n_items,
                  (void *)&nl,  (void *)&n,    (void *)&chi,      (void *)&S,        (void *)&Ibot,
                  (void *)&Itop, (void *)&I,   (void *)&flags,    (void *)&epoch,    (void *)&err,
                  (void *)&cap};
  VRT_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kern), dim3((unsigned)blocks), dim3(256), args, 0,
                                     s));
}

template <typename T, int V>
void launch_pv(hipStream_t s, const vrt::PersistItems &it, int32_t mb, const int4 *ri,
               const typename vrt::RecOf<T>::type *rf, int32_t nl, int64_t n, const T *chi, const T *S, const T *Ibot,
               const T *Itop, T *I, int32_t *flags, const int32_t *epoch, int32_t *err, int64_t cap) {
  switch (vrt::lanes_per_record(nl / V)) {
    case 64: launch_pc<T, 64, V>(s, it, mb, ri, rf, nl, n, chi, S, Ibot, Itop, I, flags, epoch, err, cap); break;
    case 32: launch_pc<T, 32, V>(s, it, mb, ri, rf, nl, n, chi, S, Ibot, Itop, I, flags, epoch, err, cap); break;
    case 16: launch_pc<T, 16, V>(s, it, mb, ri, rf, nl, n, chi, S, Ibot, Itop, I, flags, epoch, err, cap); break;
    case 8: launch_pc<T, 8, V>(s, it, mb, ri, rf, nl, n, chi, S, Ibot, Itop, I, flags, epoch, err, cap); break;
    case 4: launch_pc<T, 4, V>(s, it, mb, ri, rf, nl, n, chi, S, Ibot, Itop, I, flags, epoch, err, cap); break;
    case 2: launch_pc<T, 2, V>(s, it, mb, ri, rf, nl, n, chi, S, Ibot, Itop, I, flags, epoch, err, cap); break;
    default: launch_pc<T, 1, V>(s, it, mb, ri, rf, nl, n, chi, S, Ibot, Itop, I, flags, epoch, err, cap); break;
  }
}

}  // namespace

namespace vrt {

bool al16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

void launch_epoch(hipStream_t s, int32_t *epoch) {
  hipLaunchKernelGGL(epoch_kernel, dim3(1), dim3(1), 0, s, epoch);
  VRT_HIP(hipGetLastError());
}

int32_t persistent_records_per_wave(int32_t nl, int elem_bytes, bool aligned) {
  const int VW = 16 / elem_bytes;
  const int V = (aligned && nl % VW == 0) ? VW : 1;
  return 64 / lanes_per_record(nl / V);
}

template <typename T>
void launch_persistent_sweep(hipStream_t s, const PersistItems &items, int32_t max_blocks, const int4 *ri,
                             const typename RecOf<T>::type *rf, int32_t nl, int64_t n, const T *chi, const T *S,
                             const T *Ibot, const T *Itop, T *I, int32_t *flags, const int32_t *epoch, int32_t *err,
                             int64_t spin_cap) {
  if (items.n_items <= 0) return;
  constexpr int VW = 16 / sizeof(T);
  const bool aligned = al16(chi) && al16(S) && al16(Ibot) && al16(Itop) && al16(I);
  if (aligned && nl % VW == 0)
    launch_pv<T, VW>(s, items, max_blocks, ri, rf, nl, n, chi, S, Ibot, Itop, I, flags, epoch, err, spin_cap);
  else
    launch_pv<T, 1>(s, items, max_blocks, ri, rf, nl, n, chi, S, Ibot, Itop, I, flags, epoch, err, spin_cap);
}

template void launch_persistent_sweep<float>(hipStream_t, const PersistItems &, int32_t, const int4 *, const RecF32 *,
                                             int32_t, int64_t, const float *, const float *, const float *,
                                             const float *, float *, int32_t *, const int32_t *, int32_t *, int64_t);
template void launch_persistent_sweep<double>(hipStream_t, const PersistItems &, int32_t, const int4 *,
                                              const RecF64 *, int32_t, int64_t, const double *, const double *,
                                              const double *, const double *, double *, int32_t *, const int32_t *,
                                              int32_t *, int64_t);

}  // namespace vrt
