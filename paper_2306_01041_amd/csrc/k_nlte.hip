// Two-level-atom Lambda iteration on the GPU (Sect. 2.1, Eq. 3 and 4).
//
// Per iteration: (1) assemble the total opacity and source of every (site,
// wavelength) from the line source function S_L (double precision):
//   chi = chi_c + chi_L phi,  S = (chi_L phi S_L + chi_c B) / chi,
// stored in the sweep precision; (2) the formal solution of every ray; (3) one
// fused pass that forms the profile-weighted mean intensity
//   Jbar = sum_lambda wlam phi sum_r w_r I_r
// in double precision straight from the per-ray intensities (J per wavelength
// never goes to memory; Jbar per site does, 8 bytes), then a per-site pass
// updates S_L <- (1 - eps) Jbar + eps B in double precision and max-reduces
// |dS_L| / |S_L| for the convergence test, per atmosphere when several
// independent atmospheres are solved as one grid.

#include "segment.h"
#include "vrt_internal.h"

namespace {

// Rows of chi and S have ld >= nl entries and start cs >= ld apart (the
// iteration pairs them: S = chi + ld, cs = 2 ld); the ld - nl padding entries
// take the continuum alone (finite values the sweep may carry but nothing reads).
template <typename T>
__global__ __launch_bounds__(256) void nlte_assemble_kernel(int64_t n, int32_t nl, int32_t ld, int64_t cs,
                                                            const double *__restrict__ phi,
                                                            const double *__restrict__ chi_L,
                                                            const double *__restrict__ chi_c,
                                                            const double *__restrict__ B,
                                                            const double *__restrict__ S_L, T *__restrict__ chi,
                                                            T *__restrict__ S) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * ld) return;
  const int64_t i = t / ld;
  const int32_t l = (int32_t)(t - i * ld);
  const int64_t o = i * cs + l;
  if (l >= nl) {
    chi[o] = (T)chi_c[i];
    S[o] = (T)B[i];
    return;
  }
  const double lo = chi_L[i] * phi[i * nl + l];
  const double c = chi_c[i] + lo;
  chi[o] = (T)c;
  S[o] = (T)((lo * S_L[i] + chi_c[i] * B[i]) / c);
}

// out[i cs + l] = v[i] for l < ld
template <typename T>
__global__ void broadcast_kernel(int64_t n, int32_t ld, int64_t cs, const double *__restrict__ v,
                                 T *__restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * ld) return;
  const int64_t i = t / ld;
  out[i * cs + (t - i * ld)] = (T)v[i];
}

__global__ void zero_u64_array_kernel(int32_t count, unsigned long long *p) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = 0ull;
}

// atmosphere holding site i: the largest a with atm_ptr[a] <= i (empty
// atmospheres are skipped because a later one starts at the same offset)
__device__ __forceinline__ int32_t atm_of(int64_t i, int32_t n_atm, const int64_t *atm_ptr) {
  int32_t lo = 0, hi = n_atm - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) / 2;
    if (atm_ptr[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Profile-weighted mean intensity Jbar = sum_lambda wlam phi sum_r w_r I_r, in
// double precision. Half a wavefront (32 lanes) per site, each lane a 16-byte
// vector of wavelengths; the ray sum runs in fixed order and the wavelength
// sum is a fixed shuffle tree, so the result is deterministic. I rows have
// ld >= nl entries (ld a multiple of the vector width; only the first nl are
// line wavelengths).
template <typename T>
__global__ __launch_bounds__(256) void jbar_kernel(int64_t n, int32_t nl, int32_t ld, int32_t R,
                                                   const T *__restrict__ I, const double *__restrict__ w,
                                                   const double *__restrict__ wlam, const double *__restrict__ phi,
                                                   double *__restrict__ Jbar) {
  constexpr int V = 16 / (int)sizeof(T);
  typedef T VT __attribute__((ext_vector_type(V)));
  const int lane = threadIdx.x & 63;
  const int l32 = lane & 31;
  const int64_t site = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 2 + (lane >> 5);
  double part = 0.0;
  if (site < n) {
    const int64_t nn = n * ld;
    for (int l = l32 * V; l < nl; l += 32 * V) {
      double acc[V];
#pragma unroll
      for (int e = 0; e < V; ++e) acc[e] = 0.0;
      // rays in order, eight loads in flight before their sums (each intensity
      // is read once: non-temporal streaming loads)
      const T *Ip = I + site * ld + l;
      int32_t r = 0;
      for (; r + 8 <= R; r += 8) {
        VT x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = __builtin_nontemporal_load(reinterpret_cast<const VT *>(Ip + (int64_t)(r + u) * nn));
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const double wr = w[r + u];
#pragma unroll
          for (int e = 0; e < V; ++e) acc[e] += wr * (double)x[u][e];
        }
      }
      for (; r < R; ++r) {
        const VT x = __builtin_nontemporal_load(reinterpret_cast<const VT *>(Ip + (int64_t)r * nn));
        const double wr = w[r];
#pragma unroll
        for (int e = 0; e < V; ++e) acc[e] += wr * (double)x[e];
      }
#pragma unroll
      for (int e = 0; e < V; ++e)
        if (l + e < nl) part += wlam[l + e] * phi[site * nl + l + e] * acc[e];
    }
  }
  // xor offsets below 32 stay inside each half-wavefront
#pragma unroll
  for (int o = 16; o >= 1; o >>= 1) part += __shfl_xor(part, o, 64);
  if (site < n && l32 == 0) Jbar[site] = part;
}

// Diagonal of the line operator for the accelerated (Jacobi) iteration:
//   Lambda*_ii(lambda) = sum_r w_r sum_j w_j Psi_0(x_j),  x_j = (chi_kj + chi_i) ds_j / 2,
// the weight of S_i in I_i along each ray (Eq. 2 with linear S, Eq. 5; upwind
// intensities do not depend on S_i, boundary sites have none), and
//   Lbar_i = sum_lambda wlam phi (chi_L phi / chi) Lambda*_ii(lambda),
// the weight of S_L,i in Jbar_i (S_L enters S_lambda with chi_L phi / chi).
// Opacities chi = chi_c + chi_L phi are formed here in double precision. One
// wavefront per site, lanes over wavelengths, rays summed in fixed order.
__global__ __launch_bounds__(256) void line_diag_kernel(int64_t n, int32_t nl, int32_t R,
                                                        const double *__restrict__ ray_w,
                                                        const int32_t *__restrict__ k1,
                                                        const int32_t *__restrict__ k2,
                                                        const double *__restrict__ w1,
                                                        const double *__restrict__ ds1,
                                                        const double *__restrict__ ds2,
                                                        const double *__restrict__ chi_c,
                                                        const double *__restrict__ chi_L,
                                                        const double *__restrict__ phi,
                                                        const double *__restrict__ wlam, double *__restrict__ Lbar) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < n; i += waves) {
    double part = 0.0;
    for (int l = lane; l < nl; l += 64) {
      const double pl = phi[i * nl + l];
      const double ci = chi_c[i] + chi_L[i] * pl;
      double diag = 0.0;
      for (int32_t r = 0; r < R; ++r) {
        const int64_t ri = (int64_t)r * n + i;
        const int32_t a = k1[ri], b = k2[ri];
        if (a < 0) continue;
        double E, pu, p0;
        const double ca = chi_c[a] + chi_L[a] * phi[(int64_t)a * nl + l];
        vrt::Seg<double>::weights(0.5 * (ca + ci) * ds1[ri], E, pu, p0);
        double sum;
        if (b < 0) {
          sum = p0;
        } else {
          const double cb = chi_c[b] + chi_L[b] * phi[(int64_t)b * nl + l];
          double p0b;
          vrt::Seg<double>::weights(0.5 * (cb + ci) * ds2[ri], E, pu, p0b);
          sum = w1[ri] * p0 + (1.0 - w1[ri]) * p0b;
        }
        diag += ray_w[r] * sum;
      }
      part += wlam[l] * pl * (chi_L[i] * pl / ci) * diag;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o, 64);
    if (lane == 0) Lbar[i] = part;
  }
}

// NaN-keeping maximum of non-negative changes (a NaN must reach the host)
__device__ __forceinline__ double keep_nan_max(double m, double x) { return (x > m || x != x) ? x : m; }

// One thread per site: S_line <- (1 - eps) Jbar + eps B for sites of active
// atmospheres (with Lbar, the accelerated form S_line + [(1 - eps) Jbar + eps B
// - S_line] / [1 - (1 - eps) Lbar]), and the largest |dS|/|S| per atmosphere (a
// block covers a contiguous range of sites, hence of atmospheres; one atomic
// per block and atmosphere it touches). Inactive (converged) atmospheres keep
// their S_line.
__global__ __launch_bounds__(256) void line_update_kernel(int64_t n, const double *__restrict__ Jbar,
                                                          const double *__restrict__ B, double eps,
                                                          const double *__restrict__ Lbar,
                                                          double *__restrict__ S_L, int32_t n_atm,
                                                          const int64_t *__restrict__ atm_ptr,
                                                          const int32_t *__restrict__ active,
                                                          unsigned long long *dS_bits) {
  __shared__ double red[4];
  const int64_t b0 = (int64_t)blockIdx.x * blockDim.x;
  if (b0 >= n) return;  // uniform over the block
  const int64_t b1 = (b0 + blockDim.x < n) ? b0 + blockDim.x : n;
  const int32_t a0 = atm_of(b0, n_atm, atm_ptr), a1 = atm_of(b1 - 1, n_atm, atm_ptr);
  const int64_t i = b0 + threadIdx.x;
  int32_t a = -1;
  double d = -1.0;  // -1: no change recorded by this thread
  if (i < n) {
    a = atm_of(i, n_atm, atm_ptr);
    if (active[a]) {
      const double s_old = S_L[i];
      const double s_fs = (1.0 - eps) * Jbar[i] + eps * B[i];
      const double s_new = Lbar ? s_old + (s_fs - s_old) / (1.0 - (1.0 - eps) * Lbar[i]) : s_fs;
      d = fabs(s_new - s_old) / fabs(s_old);
      S_L[i] = s_new;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int32_t k = a0; k <= a1; ++k) {
    double m = (a == k) ? d : -1.0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = keep_nan_max(m, __shfl_xor(m, o, 64));
    if (lane == 0) red[wv] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      double mb = red[0];
      for (int q = 1; q < (int)(blockDim.x >> 6); ++q) mb = keep_nan_max(mb, red[q]);
      // non-negative doubles order like their bit patterns; NaN sorts above +inf
      if (!(mb < 0.0)) atomicMax(&dS_bits[k], (unsigned long long)__double_as_longlong(mb));
    }
    __syncthreads();
  }
}

__global__ void check_partition_kernel(int64_t n, int32_t R, const int32_t *__restrict__ k1,
                                       const int32_t *__restrict__ k2, int32_t n_atm,
                                       const int64_t *__restrict__ atm_ptr, int32_t *bad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * R) return;
  const int64_t i = t % n;
  const int32_t a = atm_of(i, n_atm, atm_ptr);
  const int64_t lo = atm_ptr[a], hi = atm_ptr[a + 1];
  const int32_t u = k1[t], v = k2[t];
  const bool out = (u >= 0 && (u < lo || u >= hi)) || (v >= 0 && (v < lo || v >= hi));
  if (out) atomicOr(bad, 1);
}

inline unsigned nb(int64_t work, int bs) { return vrt::grid_blocks(work, bs); }

}  // namespace

namespace vrt {

template <typename T>
void launch_nlte_assemble(hipStream_t s, int64_t n, int32_t nl, int32_t ld, int64_t cs, const double *phi,
                          const double *chi_L, const double *chi_c, const double *B, const double *S_L, T *chi,
                          T *S) {
  if (n * ld == 0) return;
  hipLaunchKernelGGL(nlte_assemble_kernel<T>, dim3(nb(n * ld, 256)), dim3(256), 0, s, n, nl, ld, cs, phi, chi_L,
                     chi_c, B, S_L, chi, S);
  VRT_HIP(hipGetLastError());
}

template <typename T>
void launch_broadcast(hipStream_t s, int64_t n, int32_t ld, int64_t cs, const double *v, T *out) {
  if (n * ld == 0) return;
  hipLaunchKernelGGL(broadcast_kernel<T>, dim3(nb(n * ld, 256)), dim3(256), 0, s, n, ld, cs, v, out);
  VRT_HIP(hipGetLastError());
}

void launch_zero_u64(hipStream_t s, int32_t count, unsigned long long *p) {
  if (count <= 0) return;
  hipLaunchKernelGGL(zero_u64_array_kernel, dim3(nb(count, 256)), dim3(256), 0, s, count, p);
  VRT_HIP(hipGetLastError());
}

void launch_check_partition(hipStream_t s, int64_t n, int32_t R, const int32_t *k1, const int32_t *k2, int32_t n_atm,
                            const int64_t *atm_ptr, int32_t *bad) {
  if (n * R == 0) return;
  hipLaunchKernelGGL(check_partition_kernel, dim3(nb(n * R, 256)), dim3(256), 0, s, n, R, k1, k2, n_atm, atm_ptr, bad);
  VRT_HIP(hipGetLastError());
}

template <typename T>
void launch_line_update(hipStream_t s, int64_t n, int32_t nl, int32_t ld, int32_t R, const T *I, const double *w,
                        const double *wlam, const double *phi, const double *B, double eps, double *S_L,
                        int32_t n_atm, const int64_t *atm_ptr, const int32_t *active, unsigned long long *dS_bits,
                        double *Jbar, const double *Lbar) {
  if (n == 0) return;
  if (ld % (16 / (int)sizeof(T)) != 0 || (reinterpret_cast<uintptr_t>(I) & 15u) != 0)
    throw Error(VRT_E_STATE, "line update needs 16-byte intensity rows");
  hipLaunchKernelGGL(jbar_kernel<T>, dim3(nb(n, 8)), dim3(256), 0, s, n, nl, ld, R, I, w, wlam, phi, Jbar);
  VRT_HIP(hipGetLastError());
  hipLaunchKernelGGL(line_update_kernel, dim3(nb(n, 256)), dim3(256), 0, s, n, Jbar, B, eps, Lbar, S_L, n_atm,
                     atm_ptr, active, dS_bits);
  VRT_HIP(hipGetLastError());
}

void launch_line_diag(hipStream_t s, int64_t n, int32_t nl, int32_t R, const double *ray_w, const int32_t *k1,
                      const int32_t *k2, const double *w1, const double *ds1, const double *ds2, const double *chi_c,
                      const double *chi_L, const double *phi, const double *wlam, double *Lbar) {
  if (n == 0) return;
  int64_t blocks = (n + 3) / 4;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(line_diag_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n, nl, R, ray_w, k1, k2, w1, ds1, ds2,
                     chi_c, chi_L, phi, wlam, Lbar);
  VRT_HIP(hipGetLastError());
}

template void launch_nlte_assemble<float>(hipStream_t, int64_t, int32_t, int32_t, int64_t, const double *,
                                          const double *, const double *, const double *, const double *, float *,
                                          float *);
template void launch_nlte_assemble<double>(hipStream_t, int64_t, int32_t, int32_t, int64_t, const double *,
                                           const double *, const double *, const double *, const double *, double *,
                                           double *);
template void launch_broadcast<float>(hipStream_t, int64_t, int32_t, int64_t, const double *, float *);
template void launch_broadcast<double>(hipStream_t, int64_t, int32_t, int64_t, const double *, double *);
template void launch_line_update<float>(hipStream_t, int64_t, int32_t, int32_t, int32_t, const float *,
                                        const double *, const double *, const double *, const double *, double,
                                        double *, int32_t, const int64_t *, const int32_t *, unsigned long long *,
                                        double *, const double *);
template void launch_line_update<double>(hipStream_t, int64_t, int32_t, int32_t, int32_t, const double *,
                                         const double *, const double *, const double *, const double *, double,
                                         double *, int32_t, const int64_t *, const int32_t *, unsigned long long *,
                                         double *, const double *);

}  // namespace vrt
