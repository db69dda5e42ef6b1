// Formal-solution sweep with the quadratic Bezier segment, the higher-order
// solver the paper points to for its Delaunay lines (Sect. 2.5; de la Cruz
// Rodriguez & Piskunov 2013).
//
// Along an upwind line of optical depth x from site k to site i the source is
// the quadratic Bezier curve with end values S_k, S_i and control value C:
//   I_j = e^-x I_k + alpha(x) S_k + beta(x) S_i + gamma(x) C,
//   alpha = [2 - e^-x (x^2 + 2x + 2)]/x^2, beta = 1 - 2(e^-x + x - 1)/x^2,
//   gamma = 2(x - 2 + e^-x (x + 2))/x^2,
// summed from their power series below x = 1. C = S_i - x S'_i / 2 with the
// derivative S'_i along the ray from the Fritsch-Butland harmonic mean of the
// upwind slope (S_i - S_k)/x and the downwind slope d_d, zero where the two
// differ in sign, the upwind slope alone where the site has no downwind line;
// C is kept between S_k and S_i. The downwind slope averages the site's
// downwind lines (the upwind selection of the opposite direction, Eq. 5-6):
//   d_d = sum_j q_j (S_qj - S_i)/x'_j, x_d = sum_j q_j x'_j,
//   x'_j = (chi_qj + chi_i) ds'_j / 2.
// The site's intensity is w1 I_1 + (1 - w1) I_2 (Eq. 5).
//
// One launch updates a contiguous range of the sweep records (one level of
// one ray, or one level step of all rays), 16 lanes per record striding over
// wavelengths with 16-byte vectors when the rows allow, workgroups dealt to
// the dies in contiguous chunks of records.

#include "persist.h"
#include "segment.h"
#include "vrt_internal.h"

namespace {

// a / b: IEEE division in double precision; in single precision the hardware
// reciprocal (about 1 ulp) times a
__device__ __forceinline__ double qdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

template <typename T> struct Bez;

template <> struct Bez<double> {
  static __device__ __forceinline__ void weights(double x, double &E, double &a, double &b, double &c) {
    E = exp(-x);
    if (x < 1.0) {
      // Horner over m = 22 .. 3 of (-1)^(m+1) {(m-1)(m-2), 2, 2(m-2)} x^(m-3)/m!, times x
      double sa = 0.0, sb = 0.0, sc = 0.0;
#pragma unroll
      for (int m = 22; m >= 3; --m) {
        const double f = ((m & 1) ? 1.0 : -1.0) * vrt::inv_factorial(m);
        sa = sa * x + (double)((m - 1) * (m - 2)) * f;
        sb = sb * x + 2.0 * f;
        sc = sc * x + 2.0 * (double)(m - 2) * f;
      }
      a = sa * x;
      b = sb * x;
      c = sc * x;
    } else {
      const double x2 = x * x;
      a = (2.0 - E * (x2 + 2.0 * x + 2.0)) / x2;
      b = 1.0 - 2.0 * (E + x - 1.0) / x2;
      c = 2.0 * (x - 2.0 + E * (x + 2.0)) / x2;
    }
  }
};

template <> struct Bez<float> {
  static __device__ __forceinline__ void weights(float x, float &E, float &a, float &b, float &c) {
    E = expf(-x);
    if (x < 1.0f) {
      // m = 13 .. 3: the first omitted term is below 2e-8 of each weight at x = 1
      float sa = 0.0f, sb = 0.0f, sc = 0.0f;
#pragma unroll
      for (int m = 13; m >= 3; --m) {
        const float f = (float)(((m & 1) ? 1.0 : -1.0) * vrt::inv_factorial(m));
        sa = sa * x + (float)((m - 1) * (m - 2)) * f;
        sb = sb * x + 2.0f * f;
        sc = sc * x + 2.0f * (float)(m - 2) * f;
      }
      a = sa * x;
      b = sb * x;
      c = sc * x;
    } else {
      const float x2 = x * x, r = __builtin_amdgcn_rcpf(x2);
      a = (2.0f - E * (x2 + 2.0f * x + 2.0f)) * r;
      b = 1.0f - 2.0f * (E + x - 1.0f) * r;
      c = 2.0f * (x - 2.0f + E * (x + 2.0f)) * r;
    }
  }
};

// control value of one upwind line (see the file comment)
template <typename T>
__device__ __forceinline__ T control(T Su, T S0, T x, bool has_d, T dd, T xd) {
  if (!(x > T(0))) return S0;
  const T du = qdiv(S0 - Su, x);
  T d;
  if (!has_d) {
    d = du;
  } else if (du * dd > T(0)) {
    const T a = (T(1) + qdiv(xd, x + xd)) * T(1.0 / 3.0);
    d = qdiv(du * dd, a * dd + (T(1) - a) * du);
  } else {
    d = T(0);
  }
  T C = S0 - T(0.5) * x * d;
  const T lo = Su < S0 ? Su : S0, hi = Su < S0 ? S0 : Su;
  C = C < lo ? lo : C;
  C = C > hi ? hi : C;
  return C;
}

constexpr int kLanes = 16;  // lanes per record

template <typename T, int V> struct BLane {
  typedef T type __attribute__((ext_vector_type(V)));
  static __device__ __forceinline__ type load(const T *p) { return *reinterpret_cast<const type *>(p); }
  static __device__ __forceinline__ void store(T *p, const type &v) { *reinterpret_cast<type *>(p) = v; }
};
template <typename T> struct BLane<T, 1> {
  typedef T type;
  static __device__ __forceinline__ type load(const T *p) { return *p; }
  static __device__ __forceinline__ void store(T *p, const type &v) { *p = v; }
};
template <typename T, int V> __device__ __forceinline__ T el(const typename BLane<T, V>::type &v, int k) {
  if constexpr (V == 1) return v;
  else return v[k];
}
template <typename T, int V> __device__ __forceinline__ void set_el(typename BLane<T, V>::type &v, int k, T x) {
  if constexpr (V == 1) v = x;
  else v[k] = x;
}

// Workgroup b works on the (b mod k)-th of k contiguous chunks of the launch's
// records, so neighbouring records share an accelerator die (dealt round-robin).
__device__ __forceinline__ int64_t die_chunked_block(int32_t k) {
  const int64_t b = blockIdx.x, nb = gridDim.x;
  if (k <= 1 || nb < k) return b;
  const int64_t x = b % k, j = b / k, per = nb / k, rem = nb % k;
  return x * per + (x < rem ? x : rem) + j;
}

// Intensity rows of one ray, addressed by element index within the ray's
// block: plain accesses for the level-step kernel (the kernel boundary orders
// them), device-scope buffer accesses for the persistent kernel
template <typename T, int V> struct PlainRows {
  T *base;
  __device__ __forceinline__ typename BLane<T, V>::type load(int64_t e) const { return BLane<T, V>::load(base + e); }
  __device__ __forceinline__ void store(int64_t e, const typename BLane<T, V>::type &v) const {
    BLane<T, V>::store(base + e, v);
  }
};
template <typename T, int V, bool BIG> struct CoherentRows {
  vrt_persist::RayBlock<BIG> blk;
  __device__ __forceinline__ typename BLane<T, V>::type load(int64_t e) const {
    return blk.template load<typename BLane<T, V>::type>(e * (int64_t)sizeof(T));
  }
  __device__ __forceinline__ void store(int64_t e, const typename BLane<T, V>::type &v) const {
    blk.template store<typename BLane<T, V>::type>(e * (int64_t)sizeof(T), v);
  }
};

// The quadratic-segment update of one record (site of one ray) for the
// wavelengths l0, l0 + kLanes V, ...; rows: the record's ray's intensities.
// The input rows of site i (chi, S, boundary intensities) start at i cs (cs >= nl).
template <typename T, int V, typename Rows>
__device__ __forceinline__ void bezier_record(const int4 q, const typename vrt::RecOf<T>::type *__restrict__ rf,
                                              int64_t rec, int l0, int32_t nl, int64_t cs, int64_t n,
                                              const int32_t *__restrict__ q1, const int32_t *__restrict__ q2,
                                              const double *__restrict__ qw1, const double *__restrict__ qd1,
                                              const double *__restrict__ qd2, const T *__restrict__ chi,
                                              const T *__restrict__ S, const T *__restrict__ Ibot,
                                              const T *__restrict__ Itop, const Rows &rows) {
  using L = BLane<T, V>;
  using VT = typename L::type;
  const int32_t site = q.x, k1 = q.y, k2 = q.z, ray = q.w >> 1;
  const bool up = (q.w & 1) != 0;
  const int64_t bi = (int64_t)site * nl, ei = (int64_t)site * cs;
  if (k1 < 0) {
    for (int l = l0; l < nl; l += kLanes * V) {
      VT v;
      if (up) v = L::load(Ibot + ei + l);
      else if (Itop) v = L::load(Itop + ei + l);
      else v = VT(T(0));
      rows.store(bi + l, v);
    }
    return;
  }
  const auto f = rf[rec];
  const bool two = k2 >= 0;
  const T w1 = two ? (T)f.w1 : T(1);
  const T h1 = T(0.5) * f.ds1, h2 = T(0.5) * f.ds2;
  const int64_t rs = (int64_t)ray * n + site;
  const int32_t d1 = q1[rs], d2 = q2[rs];
  const bool two_d = d2 >= 0;
  const T qa = two_d ? (T)qw1[rs] : T(1);
  const T g1 = T(0.5) * (T)qd1[rs], g2 = T(0.5) * (T)qd2[rs];
  const int64_t bk1 = (int64_t)k1 * nl, bk2 = (int64_t)(two ? k2 : k1) * nl;
  const int64_t ek1 = (int64_t)k1 * cs, ek2 = (int64_t)(two ? k2 : k1) * cs;
  const int64_t ed1 = (int64_t)(d1 >= 0 ? d1 : site) * cs, ed2 = (int64_t)(two_d ? d2 : site) * cs;
  for (int l = l0; l < nl; l += kLanes * V) {
    const VT ci = L::load(chi + ei + l), si = L::load(S + ei + l);
    const VT ck1 = L::load(chi + ek1 + l), sk1 = L::load(S + ek1 + l), ik1 = rows.load(bk1 + l);
    VT ck2 = ck1, sk2 = sk1, ik2 = ik1;
    if (two) {
      ck2 = L::load(chi + ek2 + l);
      sk2 = L::load(S + ek2 + l);
      ik2 = rows.load(bk2 + l);
    }
    VT cq1 = ci, sq1 = si, cq2 = ci, sq2 = si;
    if (d1 >= 0) {
      cq1 = L::load(chi + ed1 + l);
      sq1 = L::load(S + ed1 + l);
      if (two_d) {
        cq2 = L::load(chi + ed2 + l);
        sq2 = L::load(S + ed2 + l);
      }
    }
    VT out;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const T c0 = el<T, V>(ci, e), s0 = el<T, V>(si, e);
      bool has_d = d1 >= 0;
      T dd = T(0), xd = T(0);
      if (has_d) {
        const T x1 = (el<T, V>(cq1, e) + c0) * g1;
        const T x2 = two_d ? (el<T, V>(cq2, e) + c0) * g2 : T(1);
        if (!(x1 > T(0)) || !(x2 > T(0))) {
          has_d = false;
        } else {
          dd = qa * qdiv(el<T, V>(sq1, e) - s0, x1);
          xd = qa * x1;
          if (two_d) {
            dd += (T(1) - qa) * qdiv(el<T, V>(sq2, e) - s0, x2);
            xd += (T(1) - qa) * x2;
          }
        }
      }
      T Iv;
      {
        const T x = (el<T, V>(ck1, e) + c0) * h1;
        const T Su = el<T, V>(sk1, e);
        const T C = control(Su, s0, x, has_d, dd, xd);
        T E, a, b, c;
        Bez<T>::weights(x, E, a, b, c);
        Iv = w1 * (E * el<T, V>(ik1, e) + a * Su + b * s0 + c * C);
      }
      if (two) {
        const T x = (el<T, V>(ck2, e) + c0) * h2;
        const T Su = el<T, V>(sk2, e);
        const T C = control(Su, s0, x, has_d, dd, xd);
        T E, a, b, c;
        Bez<T>::weights(x, E, a, b, c);
        Iv += (T(1) - w1) * (E * el<T, V>(ik2, e) + a * Su + b * s0 + c * C);
      }
      set_el<T, V>(out, e, Iv);
    }
    rows.store(bi + l, out);
  }
}


// kLanes lanes per record, V consecutive wavelengths per lane (nl a multiple of V)
template <typename T, int V>
__global__ __launch_bounds__(256) void bezier_sweep_kernel(
    const int4 *__restrict__ ri, const typename vrt::RecOf<T>::type *__restrict__ rf, int64_t rec_begin,
    int64_t rec_count, int32_t nl, int64_t cs, int64_t n, const int32_t *__restrict__ q1,
    const int32_t *__restrict__ q2, const double *__restrict__ qw1, const double *__restrict__ qd1,
    const double *__restrict__ qd2, const T *__restrict__ chi, const T *__restrict__ S, const T *__restrict__ Ibot,
    const T *__restrict__ Itop, T *I, int32_t xcd_chunks) {
  const int64_t t = die_chunked_block(xcd_chunks) * blockDim.x + threadIdx.x;
  const int64_t r = t / kLanes;
  if (r >= rec_count) return;
  const int l0 = (int)(t % kLanes) * V;
  const int64_t rec = rec_begin + r;
  const int4 q = ri[rec];
  const PlainRows<T, V> rows{I + (int64_t)(q.w >> 1) * n * nl};
  bezier_record<T, V>(q, rf, rec, l0, nl, cs, n, q1, q2, qw1, qd1, qd2, chi, S, Ibot, Itop, rows);
}

// Persistent quadratic-segment sweep: every ray and level in one launch, with
// the dataflow, registration and device-scope row accesses of the persistent
// linear sweep. Items: (level step, ray) segments in step order, at most
// 64 / kLanes records each; item_cnt = record count + 256 x ray. Only the
// upwind rows pass between wavefronts (the downwind lines read S and chi).
template <typename T, int V, bool BIG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_num_sgpr(80))) void persistent_bezier_kernel(
    const int4 *__restrict__ ri, const typename vrt::RecOf<T>::type *__restrict__ rf,
    const int64_t *__restrict__ item_rec, const int32_t *__restrict__ item_cnt, int64_t n_items, int32_t nl,
    int64_t cs, int64_t n, const int32_t *__restrict__ q1, const int32_t *__restrict__ q2, const double *__restrict__ qw1,
    const double *__restrict__ qd1, const double *__restrict__ qd2, const T *__restrict__ chi,
    const T *__restrict__ S, const T *__restrict__ Ibot, const T *__restrict__ Itop, T *I, int64_t flag_ld,
    int32_t *flags, int32_t *words, int64_t spin_cap) {
  const int32_t epoch = words[0];
  int32_t *err = words + 1;
  const int lane = threadIdx.x & 63;
  int64_t W = 0;
  const int64_t rank =
      vrt_persist::register_wave(words, (int32_t)(gridDim.x * (blockDim.x >> 6)), spin_cap, lane, W);
  if (rank < 0) return;
  const int l0 = (lane % kLanes) * V;
  const int sub = lane / kLanes;
  for (int64_t item = rank; item < n_items; item += W) {
    const int32_t cr = item_cnt[item];
    const bool live = sub < (cr & 255);
    const int64_t rec = item_rec[item] + sub;
    int4 q = make_int4(0, -1, -1, 0);
    if (live) q = ri[rec];
    const int32_t site = q.x, k1 = q.y, k2 = q.z, ray = q.w >> 1;
    int32_t *fr = flags + (int64_t)ray * flag_ld;
    if (live && k1 >= 0) {
      if (vrt_persist::wait_stamp(fr + k1, epoch, err, spin_cap) && k2 >= 0)
        vrt_persist::wait_stamp(fr + k2, epoch, err, spin_cap);
    }
    if (live) {
      // the item's ray's block of n * nl values (BIG: 4 GiB or more)
      const CoherentRows<T, V, BIG> rows{
          vrt_persist::RayBlock<BIG>(I + (int64_t)(cr >> 8) * n * nl, n * nl * (int64_t)sizeof(T))};
      bezier_record<T, V>(q, rf, rec, l0, nl, cs, n, q1, q2, qw1, qd1, qd2, chi, S, Ibot, Itop, rows);
    }
    // every row store of the wave has completed before any of its stamps
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (live && (lane % kLanes) == 0)
      __hip_atomic_store(fr + site, epoch, __ATOMIC_RELAXED, vrt_persist::kXScope);
  }
}

}  // namespace

namespace vrt {

template <typename T>
void launch_bezier_sweep(hipStream_t s, const int4 *ri, const typename RecOf<T>::type *rf, int64_t rec_begin,
                         int64_t rec_count, int32_t nl, int64_t cs, int64_t n, const int32_t *q1,
                         const int32_t *q2, const double *qw1, const double *qd1, const double *qd2, const T *chi,
                         const T *S, const T *Ibot, const T *Itop, T *I, int32_t xcd_chunks) {
  if (rec_count <= 0) return;
  const unsigned blocks = (unsigned)((rec_count * kLanes + 255) / 256);
  constexpr int V = 16 / (int)sizeof(T);
  auto al = [](const void *p) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  if (nl % V == 0 && cs % V == 0 && al(chi) && al(S) && al(Ibot) && al(Itop) && al(I))
    bezier_sweep_kernel<T, V><<<blocks, 256, 0, s>>>(ri, rf, rec_begin, rec_count, nl, cs, n, q1, q2, qw1, qd1, qd2,
                                                     chi, S, Ibot, Itop, I, xcd_chunks);
  else
    bezier_sweep_kernel<T, 1><<<blocks, 256, 0, s>>>(ri, rf, rec_begin, rec_count, nl, cs, n, q1, q2, qw1, qd1, qd2,
                                                     chi, S, Ibot, Itop, I, xcd_chunks);
  VRT_HIP(hipGetLastError());
}

int32_t bezier_records_per_wave() { return 64 / kLanes; }

template <typename T>
void launch_persistent_bezier(hipStream_t s, const PersistItems &items, int32_t max_blocks, const int4 *ri,
                              const typename RecOf<T>::type *rf, int32_t nl, int64_t cs, int64_t n,
                              const int32_t *q1, const int32_t *q2, const double *qw1, const double *qd1,
                              const double *qd2, const T *chi, const T *S, const T *Ibot, const T *Itop, T *I,
                              int64_t flag_ld, int32_t *flags, int32_t *words, int64_t spin_cap) {
  if (items.n_items <= 0) return;
  if (items.spw != 64 / kLanes) throw Error(VRT_E_STATE, "persistent item table built for another record width");
  constexpr int VW = 16 / (int)sizeof(T);
  auto al = [](const void *p) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  const bool vec = nl % VW == 0 && cs % VW == 0 && al(chi) && al(S) && al(Ibot) && al(Itop) && al(I);
  auto launch = [&](auto kern) {
    int dev = 0, cus = 0, per_cu = 0;
    VRT_HIP(hipGetDevice(&dev));
    VRT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    VRT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0));
    if (per_cu < 1) throw Error(VRT_E_HIP, "persistent Bezier kernel cannot be resident");
    // any count is correct (registration gives work only to running wavefronts)
    int64_t blocks = (int64_t)cus * per_cu;
    if (blocks > (items.n_items + 3) / 4) blocks = (items.n_items + 3) / 4;
    if (max_blocks > 0) blocks = max_blocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, s, ri, rf, items.rec.as<int64_t>(),
                       items.cnt.as<int32_t>(), items.n_items, nl, cs, n, q1, q2, qw1, qd1, qd2, chi, S, Ibot, Itop,
                       I, flag_ld, flags, words, spin_cap);
    VRT_HIP(hipGetLastError());
  };
  const bool big = n * (int64_t)nl * (int64_t)sizeof(T) >= (int64_t(1) << 32);
  if (vec) big ? launch(persistent_bezier_kernel<T, VW, true>) : launch(persistent_bezier_kernel<T, VW, false>);
  else big ? launch(persistent_bezier_kernel<T, 1, true>) : launch(persistent_bezier_kernel<T, 1, false>);
}

template void launch_persistent_bezier<float>(hipStream_t, const PersistItems &, int32_t, const int4 *,
                                              const RecF32 *, int32_t, int64_t, int64_t, const int32_t *, const int32_t *,
                                              const double *, const double *, const double *, const float *,
                                              const float *, const float *, const float *, float *, int64_t,
                                              int32_t *, int32_t *, int64_t);
template void launch_persistent_bezier<double>(hipStream_t, const PersistItems &, int32_t, const int4 *,
                                               const RecF64 *, int32_t, int64_t, int64_t, const int32_t *, const int32_t *,
                                               const double *, const double *, const double *, const double *,
                                               const double *, const double *, const double *, double *, int64_t,
                                               int32_t *, int32_t *, int64_t);

template void launch_bezier_sweep<float>(hipStream_t, const int4 *, const RecF32 *, int64_t, int64_t, int32_t,
                                         int64_t, int64_t, const int32_t *, const int32_t *, const double *, const double *,
                                         const double *, const float *, const float *, const float *, const float *,
                                         float *, int32_t);
template void launch_bezier_sweep<double>(hipStream_t, const int4 *, const RecF64 *, int64_t, int64_t, int32_t,
                                          int64_t, int64_t, const int32_t *, const int32_t *, const double *, const double *,
                                          const double *, const double *, const double *, const double *,
                                          const double *, double *, int32_t);

}  // namespace vrt
