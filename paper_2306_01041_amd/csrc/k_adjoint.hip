// Reverse (adjoint) sweep of the Voronoi formal solution and the chain rule of
// the grey LTE continuum, for gradients of a misfit with respect to per-site
// temperature and density.
//
// Forward, per ray and site i (Sect. 2.1 Eq. 2, Sect. 2.5 Eq. 5):
//   I_i = sum_j w_j (E_j I_kj + Psi_u,j S_kj + Psi_0,j S_i),  x_j = (chi_kj + chi_i) ds_j / 2.
// Reverse, in gather form: the adjoint intensity of site k collects from every
// site d that read k in the forward sweep (its dependents, listed per ray):
//   Ibar_k = seed_k + sum_d a_d E_d,          a_d = Ibar_d w_d
//   Sbar_k = sum_d a_d Psi_u,d + sum_own_j Ibar_k w_j Psi_0,j
//   chibar_k = sum_d a_d (-E_d I_k + Psi_u,d' S_k + Psi_0,d' S_d) ds_d / 2
//            + sum_own_j Ibar_k w_j (-E_j I_kj + Psi_u,j' S_kj + Psi_0,j' S_k) ds_j / 2
// (the brackets are evaluated in the cancellation-free form of dI_dx below).
// Dependents sit at higher levels, so walking the level steps downwards makes
// every Ibar_d final before it is read; each site writes only its own entries
// (no atomics, deterministic). Per-ray contributions are summed over rays in
// double precision afterwards; at boundary sites Ibar is the sensitivity to the
// boundary intensity.

#include "persist.h"
#include "segment.h"
#include "vrt_internal.h"

namespace {

template <typename T, int V> struct ALane {
  typedef T type __attribute__((ext_vector_type(V)));
  static __device__ __forceinline__ type load(const T *p) { return *reinterpret_cast<const type *>(p); }
  static __device__ __forceinline__ void store(T *p, const type &v) { *reinterpret_cast<type *>(p) = v; }
  static __device__ __forceinline__ T get(const type &v, int k) { return v[k]; }
  static __device__ __forceinline__ void set(type &v, int k, T x) { v[k] = x; }
};
template <typename T> struct ALane<T, 1> {
  typedef T type;
  static __device__ __forceinline__ type load(const T *p) { return *p; }
  static __device__ __forceinline__ void store(T *p, const type &v) { *p = v; }
  static __device__ __forceinline__ T get(const type &v, int) { return v; }
  static __device__ __forceinline__ void set(type &v, int, T x) { v = x; }
};

// Derivative of one segment's intensity I = E I_u + Psi_u S_u + Psi_0 S_d with
// respect to its optical depth x. With Psi_u' = E - Psi_0' (Psi_u + Psi_0 =
// 1 - E) it is -E (I_u - S_u) + Psi_0' (S_d - S_u): no cancellation where
// the intensity has thermalised (I_u ~ S_u ~ S_d), and the differences and
// products are formed in double precision from the stored values.
template <typename T>
__device__ __forceinline__ T dI_dx(T E, T dp0, T Iu, T Su, T Sd) {
  const double dI = (double)Iu - (double)Su, dS = (double)Sd - (double)Su;
  return (T)(-(double)E * dI + (double)dp0 * dS);
}

// Adjoint rows of one ray, addressed by element index within the ray's block:
// plain accesses for the level-step kernel (the kernel boundary orders them)
template <typename T, int V> struct PlainRows {
  T *base;
  __device__ __forceinline__ typename ALane<T, V>::type load(int64_t e) const { return ALane<T, V>::load(base + e); }
  __device__ __forceinline__ void store(int64_t e, const typename ALane<T, V>::type &v) const {
    ALane<T, V>::store(base + e, v);
  }
};

// and device-scope buffer accesses for the persistent kernel (other
// wavefronts read the rows during the launch)
template <typename T, int V, bool BIG> struct CoherentRows {
  vrt_persist::RayBlock<BIG> blk;
  __device__ __forceinline__ typename ALane<T, V>::type load(int64_t e) const {
    return blk.template load<typename ALane<T, V>::type>(e * (int64_t)sizeof(T));
  }
  __device__ __forceinline__ void store(int64_t e, const typename ALane<T, V>::type &v) const {
    blk.template store<typename ALane<T, V>::type>(e * (int64_t)sizeof(T), v);
  }
};

// The reverse update of one record (site k of one ray) for the wavelengths
// l0, l0 + C V, ...: gather from the dependents, then the own segments.
// Rows: the adjoint rows of the record's ray (dependents read, own written).
// With CK the forward rows come from checkpoint buffers (see ck_rows) instead
// of I at the site's index.
template <typename T, int C, int V, typename Rows, bool CK = false>
__device__ __forceinline__ void reverse_record(const int4 q, const typename vrt::RecOf<T>::type *__restrict__ rf,
                                               int64_t rec, int l0, int32_t nl, int64_t n, int32_t ray0,
                                               const int64_t *__restrict__ dep_ptr,
                                               const int32_t *__restrict__ dep_site,
                                               const typename vrt::RecOf<T>::type *__restrict__ dep_rec,
                                               const T *__restrict__ chi, const T *__restrict__ S,
                                               const T *__restrict__ I, const T *__restrict__ gI,
                                               const T *__restrict__ gJ, const double *__restrict__ ray_w,
                                               const Rows &rows, T *__restrict__ Sbar, T *__restrict__ Cbar,
                                               const int4 *__restrict__ ck = nullptr, const T *Ich = nullptr,
                                               const T *Ifr = nullptr) {
  using L = ALane<T, V>;
  using VT = typename L::type;
  const int32_t k = q.x, k1 = q.y, k2 = q.z, ray = q.w >> 1;
  const int64_t nn = n * nl;
  const int64_t loc = (int64_t)(ray - ray0) * nn;  // this ray in the group scratch
  const int64_t bk = (int64_t)k * nl;
  // the forward rows of the site and of its two upwind sites
  const T *Iown, *Iup1, *Iup2;
  if constexpr (CK) {
    const int4 t = ck[rec];
    Iown = Ich + (int64_t)t.x * nl;
    Iup1 = t.z >= 0 ? Ich + (int64_t)t.z * nl : Ifr + (int64_t)(-t.z - 1) * nl;
    Iup2 = t.w >= 0 ? Ich + (int64_t)t.w * nl : Ifr + (int64_t)(-t.w - 1) * nl;
  } else {
    const T *Ir = I + loc;
    Iown = Ir + bk;
    Iup1 = Ir + (int64_t)(k1 >= 0 ? k1 : 0) * nl;
    Iup2 = Ir + (int64_t)(k2 >= 0 ? k2 : 0) * nl;
  }
  const int64_t d0 = dep_ptr[(int64_t)ray * (n + 1) + k], d1 = dep_ptr[(int64_t)ray * (n + 1) + k + 1];
  const T wr = (T)ray_w[ray];
  const bool own = k1 >= 0;
  typename vrt::RecOf<T>::type f{};
  if (own) f = rf[rec];
  const bool two = k2 >= 0;
  const T w1 = two ? (T)f.w1 : T(1), w2 = T(1) - (T)f.w1;
  for (int l = l0; l < nl; l += C * V) {
    const VT ck_ = L::load(chi + bk + l), sk = L::load(S + bk + l), ik = L::load(Iown + l);
    // the seed: dL/dI of this (ray, site) plus w_r dL/dJ (whole vectors: the
    // launch takes V > 1 only when both are 16-byte aligned)
    VT ib = VT(T(0)), sb = VT(T(0)), cb = VT(T(0));
    if (gI) ib = L::load(gI + (int64_t)ray * nn + bk + l);
    if (gJ) {
      const VT j = L::load(gJ + bk + l);
#pragma unroll
      for (int e = 0; e < V; ++e) L::set(ib, e, L::get(ib, e) + wr * L::get(j, e));
    }
    // gather from the dependents
    for (int64_t t = d0; t < d1; ++t) {
      const int32_t d = dep_site[t];
      const auto dr = dep_rec[t];  // w1 = weight of the line d reads from k, ds1 = its length
      const T wd = dr.w1, hd = T(0.5) * dr.ds1;
      const int64_t bd = (int64_t)d * nl;
      const VT cd = L::load(chi + bd + l), sd = L::load(S + bd + l), ad_ = rows.load(bd + l);
#pragma unroll
      for (int e = 0; e < V; ++e) {
        T E, pu, p0, dp0;
        vrt::Seg<T>::weights((L::get(ck_, e) + L::get(cd, e)) * hd, E, pu, p0, dp0);
        const T a = L::get(ad_, e) * wd;
        L::set(ib, e, L::get(ib, e) + a * E);
        L::set(sb, e, L::get(sb, e) + a * pu);
        const T xb = a * dI_dx(E, dp0, L::get(ik, e), L::get(sk, e), L::get(sd, e));
        L::set(cb, e, L::get(cb, e) + xb * hd);
      }
    }
    // own segments (the lines k read from in the forward sweep)
    if (own) {
      for (int j = 0; j < (two ? 2 : 1); ++j) {
        const int32_t u = j == 0 ? k1 : k2;
        const T w = j == 0 ? w1 : w2;
        const T h = T(0.5) * (j == 0 ? (T)f.ds1 : (T)f.ds2);
        const int64_t bu = (int64_t)u * nl;
        const VT cu = L::load(chi + bu + l), su = L::load(S + bu + l), iu = L::load((j == 0 ? Iup1 : Iup2) + l);
#pragma unroll
        for (int e = 0; e < V; ++e) {
          T E, pu, p0, dp0;
          vrt::Seg<T>::weights((L::get(cu, e) + L::get(ck_, e)) * h, E, pu, p0, dp0);
          const T a = L::get(ib, e) * w;
          L::set(sb, e, L::get(sb, e) + a * p0);
          const T xb = a * dI_dx(E, dp0, L::get(iu, e), L::get(su, e), L::get(sk, e));
          L::set(cb, e, L::get(cb, e) + xb * h);
        }
      }
    }
    rows.store(bk + l, ib);
    L::store(Sbar + loc + bk + l, sb);
    L::store(Cbar + loc + bk + l, cb);
  }
}

// Level-step reverse kernel: one launch per level step (in decreasing order),
// C lanes per record, V wavelengths per lane. Scratch arrays (I, Ibar, Sbar,
// Cbar) hold the rays [ray0, ray0 + group) of the current ray group; with CK
// the forward rows come from the checkpoint buffers Ich and Ifr through ck.
template <typename T, int C, int V, bool CK>
__global__ __launch_bounds__(256) void reverse_kernel(
    const int4 *__restrict__ ri, const typename vrt::RecOf<T>::type *__restrict__ rf, int64_t rec_begin,
    int64_t rec_count, int32_t nl, int64_t n, int32_t ray0, const int64_t *__restrict__ dep_ptr,
    const int32_t *__restrict__ dep_site, const typename vrt::RecOf<T>::type *__restrict__ dep_rec,
    const T *__restrict__ chi, const T *__restrict__ S, const T *__restrict__ I, const T *__restrict__ gI,
    const T *__restrict__ gJ, const double *__restrict__ ray_w, T *Ibar, T *__restrict__ Sbar,
    T *__restrict__ Cbar, const int4 *__restrict__ ck, const T *Ich, const T *Ifr) {
  constexpr int SPW = 64 / C;
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t rec = wave * SPW + lane / C;
  const int l0 = (lane % C) * V;
  if (rec >= rec_count) return;
  const int4 q = ri[rec_begin + rec];
  const PlainRows<T, V> rows{Ibar + (int64_t)((q.w >> 1) - ray0) * n * nl};
  reverse_record<T, C, V, PlainRows<T, V>, CK>(q, rf, rec_begin + rec, l0, nl, n, ray0, dep_ptr, dep_site, dep_rec,
                                               chi, S, I, gI, gJ, ray_w, rows, Sbar, Cbar, ck, Ich, Ifr);
}

// Persistent reverse kernel: every level step of a ray group in one launch, the
// dataflow of the persistent forward sweep run backwards. Items are the
// group's (level step, ray) segments in decreasing step order, cut into at
// most 64/C records; item_cnt holds the record count + 256 x (ray - ray0).
// Before updating site k a lane waits until every dependent of k (the sites
// that read k in the forward sweep, all in later forward steps, so in earlier
// items) carries the epoch stamp; after writing k's adjoint row the wave
// stamps k. The adjoint rows pass between wavefronts with the device-scope
// policy; Sbar and Cbar are read only after the launch.
template <typename T, int C, int V, bool BIG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_num_sgpr(80))) void persistent_reverse_kernel(
    const int4 *__restrict__ ri, const typename vrt::RecOf<T>::type *__restrict__ rf,
    const int64_t *__restrict__ item_rec, const int32_t *__restrict__ item_cnt, int64_t n_items, int32_t nl,
    int64_t n, int32_t ray0, const int64_t *__restrict__ dep_ptr, const int32_t *__restrict__ dep_site,
    const typename vrt::RecOf<T>::type *__restrict__ dep_rec, const T *__restrict__ chi, const T *__restrict__ S,
    const T *__restrict__ I, const T *__restrict__ gI, const T *__restrict__ gJ, const double *__restrict__ ray_w,
    T *Ibar, T *__restrict__ Sbar, T *__restrict__ Cbar, int64_t flag_ld, int32_t *flags, int32_t *words,
    int64_t spin_cap) {
  const int32_t epoch = words[0];
  int32_t *err = words + 1;
  const int lane = threadIdx.x & 63;
  int64_t W = 0;
  const int64_t rank =
      vrt_persist::register_wave(words, (int32_t)(gridDim.x * (blockDim.x >> 6)), spin_cap, lane, W);
  if (rank < 0) return;
  const int l0 = (lane % C) * V;
  const int sub = lane / C;
  const int64_t nn = n * nl;
  for (int64_t item = rank; item < n_items; item += W) {
    const int32_t cr = item_cnt[item];
    const bool live = sub < (cr & 255);
    const int64_t rec = item_rec[item] + sub;
    int4 q = make_int4(0, -1, -1, 0);
    if (live) q = ri[rec];
    const int32_t k = q.x, ray = q.w >> 1;
    int32_t *fr = flags + (int64_t)ray * flag_ld;
    if (live) {
      const int64_t d0 = dep_ptr[(int64_t)ray * (n + 1) + k], d1 = dep_ptr[(int64_t)ray * (n + 1) + k + 1];
      bool ok = true;
      for (int64_t t = d0; t < d1 && ok; ++t) ok = vrt_persist::wait_stamp(fr + dep_site[t], epoch, err, spin_cap);
      // the item's ray's block of the group's adjoint rows (BIG: 4 GiB or more)
      const CoherentRows<T, V, BIG> rows{
          vrt_persist::RayBlock<BIG>(Ibar + (int64_t)(cr >> 8) * nn, nn * (int64_t)sizeof(T))};
      reverse_record<T, C, V>(q, rf, rec, l0, nl, n, ray0, dep_ptr, dep_site, dep_rec, chi, S, I, gI, gJ, ray_w,
                              rows, Sbar, Cbar);
    }
    // every adjoint-row store of the wave has completed before any of its stamps
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (live && (lane % C) == 0) __hip_atomic_store(fr + k, epoch, __ATOMIC_RELAXED, vrt_persist::kXScope);
  }
}

// Sum a ray group's contributions into double accumulators: chi, S, and the
// boundary sensitivities (Ibar at a ray's upwind-boundary sites).
template <typename T>
__global__ __launch_bounds__(256) void reverse_reduce_kernel(int64_t n, int32_t nl, int32_t ray0, int32_t group,
                                                             const double *__restrict__ dirs,
                                                             const uint8_t *__restrict__ wall,
                                                             const T *__restrict__ Ibar, const T *__restrict__ Sbar,
                                                             const T *__restrict__ Cbar, double *__restrict__ acc_chi,
                                                             double *__restrict__ acc_S, double *__restrict__ acc_Ib,
                                                             double *__restrict__ acc_It) {
  const int64_t nn = n * nl;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nn; t += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t wf = wall[t / nl];
    double c = 0.0, s = 0.0, b = 0.0, tp = 0.0;
    for (int32_t g = 0; g < group; ++g) {
      const int64_t q = (int64_t)g * nn + t;
      c += (double)Cbar[q];
      s += (double)Sbar[q];
      const bool up = dirs[3 * (ray0 + g) + 2] > 0.0;
      if (up && (wf & 1)) b += (double)Ibar[q];
      if (!up && (wf & 2)) tp += (double)Ibar[q];
    }
    acc_chi[t] += c;
    acc_S[t] += s;
    acc_Ib[t] += b;
    acc_It[t] += tp;
  }
}

template <typename T>
__global__ void to_prec_kernel(int64_t nn, const double *__restrict__ a, T *__restrict__ out) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nn; t += (int64_t)gridDim.x * blockDim.x)
    out[t] = (T)a[t];
}

// adjoint of the emergent gather: dL/dI at the emergent rows, zero elsewhere
template <typename T>
__global__ void emergent_scatter_kernel(int64_t total, int32_t nl, int64_t n, const int32_t *__restrict__ em_ray,
                                        const int32_t *__restrict__ em_site, const T *__restrict__ g_em,
                                        T *__restrict__ gI) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total * nl) return;
  const int64_t e = t / nl;
  const int32_t l = (int32_t)(t - e * nl);
  gI[((int64_t)em_ray[e] * n + em_site[e]) * nl + l] = g_em[t];
}

template <typename T> __global__ void fill_kernel(int64_t count, T *__restrict__ p) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
    p[t] = T(0);
}

// SI 2019 exact values
constexpr double kH = 6.62607015e-34;
constexpr double kC = 299792458.0;
constexpr double kK = 1.380649e-23;

// one wavefront per site, lanes over wavelengths: dL/dT and dL/drho through
// chi = kappa0 rho^2 T^9 (dchi/dT = 9 chi/T, dchi/drho = 2 chi/rho) and
// S = I_bottom = B_lambda(T), with dB/dT = B (u/T) e^u / (e^u - 1), u = hc/(lambda k T)
template <typename T>
__global__ __launch_bounds__(256) void lte_vjp_kernel(int64_t n, int32_t nl, const double *__restrict__ lam,
                                                      double kappa0, const double *__restrict__ Tk,
                                                      const double *__restrict__ rho, const T *__restrict__ g_chi,
                                                      const T *__restrict__ g_S, const T *__restrict__ g_Ib,
                                                      double *__restrict__ g_T, double *__restrict__ g_rho) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n) return;
  const double Ti = Tk[i], ri = rho[i];
  const double T3 = Ti * Ti * Ti;
  const double c = kappa0 * (ri * ri) * (T3 * T3 * T3);
  double gt = 0.0, gr = 0.0;
  for (int l = lane; l < nl; l += 64) {
    const int64_t q = i * nl + l;
    const double la = lam[l];
    const double u = (kH * kC) / (la * (kK * Ti));
    const double l2 = la * la;
    const double B = (2.0 * kH * kC * kC) / (l2 * l2 * la) / expm1(u) * 1.0e-12;
    const double dB = B * (u / Ti) * exp(u) / expm1(u);
    const double gc = (double)g_chi[q];
    gt += gc * 9.0 * c / Ti + ((double)g_S[q] + (g_Ib ? (double)g_Ib[q] : 0.0)) * dB;
    gr += gc * 2.0 * c / ri;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    gt += __shfl_xor(gt, o, 64);
    gr += __shfl_xor(gr, o, 64);
  }
  if (lane == 0) {
    g_T[i] = gt;
    g_rho[i] = gr;
  }
}

template <typename T, int C, int V>
void launch_rc(hipStream_t s, const int4 *ri, const typename vrt::RecOf<T>::type *rf, int64_t b, int64_t c, int32_t nl,
               int64_t n, int32_t ray0, const int64_t *dp, const int32_t *ds_, const typename vrt::RecOf<T>::type *dr,
               const T *chi, const T *S, const T *I, const T *gI, const T *gJ, const double *w, T *Ib, T *Sb, T *Cb,
               const int4 *ck, const T *Ich, const T *Ifr) {
  constexpr int SPW = 64 / C;
  const int64_t waves = (c + SPW - 1) / SPW;
  auto kern = ck ? reverse_kernel<T, C, V, true> : reverse_kernel<T, C, V, false>;
  hipLaunchKernelGGL(kern, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, ri, rf, b, c, nl, n, ray0, dp, ds_, dr,
                     chi, S, I, gI, gJ, w, Ib, Sb, Cb, ck, Ich, Ifr);
}

template <typename T, int V>
void launch_rv(hipStream_t s, const int4 *ri, const typename vrt::RecOf<T>::type *rf, int64_t b, int64_t c, int32_t nl,
               int64_t n, int32_t ray0, const int64_t *dp, const int32_t *ds_, const typename vrt::RecOf<T>::type *dr,
               const T *chi, const T *S, const T *I, const T *gI, const T *gJ, const double *w, T *Ib, T *Sb, T *Cb,
               const int4 *ck, const T *Ich, const T *Ifr) {
#define VRT_RC(CC) launch_rc<T, CC, V>(s, ri, rf, b, c, nl, n, ray0, dp, ds_, dr, chi, S, I, gI, gJ, w, Ib, Sb, Cb, ck, Ich, Ifr)
  switch (vrt::lanes_per_record(nl / V)) {
    case 64: VRT_RC(64); break;
    case 32: VRT_RC(32); break;
    case 16: VRT_RC(16); break;
    case 8: VRT_RC(8); break;
    case 4: VRT_RC(4); break;
    case 2: VRT_RC(2); break;
    default: VRT_RC(1); break;
  }
#undef VRT_RC
}

inline unsigned nbk(int64_t work, int bs) { return vrt::grid_blocks(work, bs); }

template <typename T, int C, int V>
void launch_prc(hipStream_t s, const vrt::PersistItems &it, int32_t max_blocks, const int4 *ri,
                const typename vrt::RecOf<T>::type *rf, int32_t nl, int64_t n, int32_t ray0, const int64_t *dp,
                const int32_t *ds_, const typename vrt::RecOf<T>::type *dr, const T *chi, const T *S, const T *I,
                const T *gI, const T *gJ, const double *w, T *Ib, T *Sb, T *Cb, int64_t flag_ld, int32_t *flags,
                int32_t *words, int64_t cap) {
  if (it.spw != 64 / C) throw vrt::Error(VRT_E_STATE, "persistent item table built for another record width");
  const bool big = n * (int64_t)nl * (int64_t)sizeof(T) >= (int64_t(1) << 32);
  auto kern = big ? persistent_reverse_kernel<T, C, V, true> : persistent_reverse_kernel<T, C, V, false>;
  int dev = 0, cus = 0, per_cu = 0;
  VRT_HIP(hipGetDevice(&dev));
  VRT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  VRT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0));
  if (per_cu < 1) throw vrt::Error(VRT_E_HIP, "persistent reverse kernel cannot be resident");
  // as for the forward persistent sweep: any count is correct
  int64_t blocks = (int64_t)cus * per_cu;
  if (blocks > (it.n_items + 3) / 4) blocks = (it.n_items + 3) / 4;
  if (max_blocks > 0) blocks = max_blocks;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, s, ri, rf, it.rec.as<int64_t>(),
                     it.cnt.as<int32_t>(), it.n_items, nl, n, ray0, dp, ds_, dr, chi, S, I, gI, gJ, w, Ib, Sb, Cb,
                     flag_ld, flags, words, cap);
  VRT_HIP(hipGetLastError());
}

template <typename T, int V>
void launch_prv(hipStream_t s, const vrt::PersistItems &it, int32_t mb, const int4 *ri,
                const typename vrt::RecOf<T>::type *rf, int32_t nl, int64_t n, int32_t ray0, const int64_t *dp,
                const int32_t *ds_, const typename vrt::RecOf<T>::type *dr, const T *chi, const T *S, const T *I,
                const T *gI, const T *gJ, const double *w, T *Ib, T *Sb, T *Cb, int64_t fl, int32_t *flags,
                int32_t *words, int64_t cap) {
#define VRT_PRC(CC)                                                                                                  \
  launch_prc<T, CC, V>(s, it, mb, ri, rf, nl, n, ray0, dp, ds_, dr, chi, S, I, gI, gJ, w, Ib, Sb, Cb, fl, flags,    \
                       words, cap)
  switch (vrt::lanes_per_record(nl / V)) {
    case 64: VRT_PRC(64); break;
    case 32: VRT_PRC(32); break;
    case 16: VRT_PRC(16); break;
    case 8: VRT_PRC(8); break;
    case 4: VRT_PRC(4); break;
    case 2: VRT_PRC(2); break;
    default: VRT_PRC(1); break;
  }
#undef VRT_PRC
}

// Forward rows of the last solution in the reverse sweep's precision: |src|
// for sign-encoded rows; NaN everywhere if a persistent sweep raised an error
// (its rows are then not all of one epoch).
template <typename Tin, typename Tout>
__global__ void rows_convert_kernel(const Tin *__restrict__ src, bool abs, Tout *__restrict__ dst, int64_t count,
                                    const int32_t *err) {
  const bool bad = err && *err != 0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
    const Tin x = src[t];
    // (a float widens to double exactly; a double rounds once to the output)
    dst[t] = bad ? (Tout)__builtin_nan("") : (Tout)(abs ? __builtin_fabs((double)x) : (double)x);
  }
}

}  // namespace

namespace vrt {

template <typename T>
void launch_reverse(hipStream_t s, const int4 *ri, const typename RecOf<T>::type *rf, int64_t rec_begin,
                    int64_t rec_count, int32_t nl, int64_t n, int32_t ray0, const int64_t *dep_ptr,
                    const int32_t *dep_site, const typename RecOf<T>::type *dep_rec, const T *chi, const T *S,
                    const T *I, const T *gI, const T *gJ, const double *ray_w, T *Ibar, T *Sbar, T *Cbar,
                    const int4 *ck, const T *Ich, const T *Ifr) {
  if (rec_count <= 0) return;
  constexpr int VW = 16 / sizeof(T);
  const bool aligned = al16(chi) && al16(S) && al16(I) && al16(gI) && al16(gJ) && al16(Ibar) && al16(Sbar) &&
                       al16(Cbar) && al16(Ich) && al16(Ifr);
  if (aligned && nl % VW == 0)
    launch_rv<T, VW>(s, ri, rf, rec_begin, rec_count, nl, n, ray0, dep_ptr, dep_site, dep_rec, chi, S, I, gI, gJ,
                     ray_w, Ibar, Sbar, Cbar, ck, Ich, Ifr);
  else
    launch_rv<T, 1>(s, ri, rf, rec_begin, rec_count, nl, n, ray0, dep_ptr, dep_site, dep_rec, chi, S, I, gI, gJ,
                    ray_w, Ibar, Sbar, Cbar, ck, Ich, Ifr);
  VRT_HIP(hipGetLastError());
}

template <typename T>
void launch_rows_convert(hipStream_t s, const void *src, bool src_f32, bool abs, T *dst, int64_t count,
                         const int32_t *err) {
  if (count <= 0) return;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (src_f32)
    hipLaunchKernelGGL((rows_convert_kernel<float, T>), dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const float *>(src), abs, dst, count, err);
  else
    hipLaunchKernelGGL((rows_convert_kernel<double, T>), dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const double *>(src), abs, dst, count, err);
  VRT_HIP(hipGetLastError());
}
template void launch_rows_convert<float>(hipStream_t, const void *, bool, bool, float *, int64_t, const int32_t *);
template void launch_rows_convert<double>(hipStream_t, const void *, bool, bool, double *, int64_t, const int32_t *);

int32_t reverse_records_per_wave(int32_t nl, int elem_bytes, bool aligned) {
  const int VW = 16 / elem_bytes;
  const int V = (aligned && nl % VW == 0) ? VW : 1;
  return 64 / lanes_per_record(nl / V);
}

template <typename T>
void launch_persistent_reverse(hipStream_t s, const PersistItems &items, int32_t max_blocks, const int4 *ri,
                               const typename RecOf<T>::type *rf, int32_t nl, int64_t n, int32_t ray0,
                               const int64_t *dep_ptr, const int32_t *dep_site, const typename RecOf<T>::type *dep_rec,
                               const T *chi, const T *S, const T *I, const T *gI, const T *gJ, const double *ray_w,
                               T *Ibar, T *Sbar, T *Cbar, int64_t flag_ld, int32_t *flags, int32_t *words,
                               int64_t spin_cap) {
  if (items.n_items <= 0) return;
  constexpr int VW = 16 / sizeof(T);
  const bool aligned = al16(chi) && al16(S) && al16(I) && al16(gI) && al16(gJ) && al16(Ibar) && al16(Sbar) &&
                       al16(Cbar);
  if (aligned && nl % VW == 0)
    launch_prv<T, VW>(s, items, max_blocks, ri, rf, nl, n, ray0, dep_ptr, dep_site, dep_rec, chi, S, I, gI, gJ, ray_w,
                      Ibar, Sbar, Cbar, flag_ld, flags, words, spin_cap);
  else
    launch_prv<T, 1>(s, items, max_blocks, ri, rf, nl, n, ray0, dep_ptr, dep_site, dep_rec, chi, S, I, gI, gJ, ray_w,
                     Ibar, Sbar, Cbar, flag_ld, flags, words, spin_cap);
}

template <typename T>
void launch_reverse_reduce(hipStream_t s, int64_t n, int32_t nl, int32_t ray0, int32_t group, const double *dirs,
                           const uint8_t *wall, const T *Ibar, const T *Sbar, const T *Cbar, double *acc_chi,
                           double *acc_S, double *acc_Ib, double *acc_It) {
  const int64_t nn = n * nl;
  if (nn == 0) return;
  int64_t blocks = (nn + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(reverse_reduce_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, n, nl, ray0, group, dirs, wall,
                     Ibar, Sbar, Cbar, acc_chi, acc_S, acc_Ib, acc_It);
  VRT_HIP(hipGetLastError());
}

template <typename T> void launch_to_prec(hipStream_t s, int64_t nn, const double *a, T *out) {
  if (nn == 0 || !out) return;
  hipLaunchKernelGGL(to_prec_kernel<T>, dim3((unsigned)std::min<int64_t>((nn + 255) / 256, 65536)), dim3(256), 0, s, nn, a, out);
  VRT_HIP(hipGetLastError());
}

template <typename T> void launch_fill_zero(hipStream_t s, int64_t count, T *p) {
  if (count == 0) return;
  hipLaunchKernelGGL(fill_kernel<T>, dim3((unsigned)std::min<int64_t>((count + 255) / 256, 65536)), dim3(256), 0, s, count, p);
  VRT_HIP(hipGetLastError());
}

template <typename T>
void launch_emergent_scatter(hipStream_t s, int64_t total, int32_t nl, int64_t n, const int32_t *em_ray,
                             const int32_t *em_site, const T *g_em, T *gI) {
  if (total * nl == 0) return;
  hipLaunchKernelGGL(emergent_scatter_kernel<T>, dim3(nbk(total * nl, 256)), dim3(256), 0, s, total, nl, n, em_ray,
                     em_site, g_em, gI);
  VRT_HIP(hipGetLastError());
}

template <typename T>
void launch_lte_vjp(hipStream_t s, int64_t n, int32_t nl, const double *lam, double kappa0, const double *T_,
                    const double *rho, const T *g_chi, const T *g_S, const T *g_Ib, double *g_T, double *g_rho) {
  if (n == 0) return;
  hipLaunchKernelGGL(lte_vjp_kernel<T>, dim3(nbk(n, 4)), dim3(256), 0, s, n, nl, lam, kappa0, T_, rho, g_chi, g_S,
                     g_Ib, g_T, g_rho);
  VRT_HIP(hipGetLastError());
}

#define VRT_INST(T)                                                                                                   \
  template void launch_reverse<T>(hipStream_t, const int4 *, const RecOf<T>::type *, int64_t, int64_t, int32_t,      \
                                  int64_t, int32_t, const int64_t *, const int32_t *, const RecOf<T>::type *,         \
                                  const T *, const T *, const T *, const T *, const T *, const double *, T *, T *,    \
                                  T *, const int4 *, const T *, const T *);                                           \
  template void launch_persistent_reverse<T>(                                                                         \
      hipStream_t, const PersistItems &, int32_t, const int4 *, const RecOf<T>::type *, int32_t, int64_t, int32_t,    \
      const int64_t *, const int32_t *, const RecOf<T>::type *, const T *, const T *, const T *, const T *, const T *, \
      const double *, T *, T *, T *, int64_t, int32_t *, int32_t *, int64_t);                                          \
  template void launch_reverse_reduce<T>(hipStream_t, int64_t, int32_t, int32_t, int32_t, const double *,             \
                                         const uint8_t *, const T *, const T *, const T *, double *, double *,        \
                                         double *, double *);                                                         \
  template void launch_to_prec<T>(hipStream_t, int64_t, const double *, T *);                                        \
  template void launch_fill_zero<T>(hipStream_t, int64_t, T *);                                                       \
  template void launch_emergent_scatter<T>(hipStream_t, int64_t, int32_t, int64_t, const int32_t *, const int32_t *, \
                                           const T *, T *);                                                           \
  template void launch_lte_vjp<T>(hipStream_t, int64_t, int32_t, const double *, double, const double *,             \
                                  const double *, const T *, const T *, const T *, double *, double *);
VRT_INST(float)
VRT_INST(double)
#undef VRT_INST

}  // namespace vrt
