// Two-level-atom Lambda iteration on the GPU (Sect. 2.1, Eq. 3 and 4).
//
// Per iteration: (1) assemble the total opacity and source of every (site,
// wavelength) from the line source function S_L (double precision):
//   chi = chi_c + chi_L phi,  S = (chi_L phi S_L + chi_c B) / chi,
// stored in the sweep precision; (2) the formal solution of every ray; (3) one
// fused pass that forms the profile-weighted mean intensity
//   Jbar = sum_lambda wlam phi sum_r w_r I_r
// in double precision straight from the per-ray intensities (J per wavelength
// never goes to memory), updates S_L <- (1 - eps) Jbar + eps B in double
// precision and max-reduces |dS_L| / |S_L| for the convergence test.

#include "vrt_internal.h"

namespace {

template <typename T>
__global__ __launch_bounds__(256) void nlte_assemble_kernel(int64_t n, int32_t nl, const double *__restrict__ phi,
                                                            const double *__restrict__ chi_L,
                                                            const double *__restrict__ chi_c,
                                                            const double *__restrict__ B,
                                                            const double *__restrict__ S_L, T *__restrict__ chi,
                                                            T *__restrict__ S) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nl) return;
  const int64_t i = t / nl;
  const double lo = chi_L[i] * phi[t];
  const double c = chi_c[i] + lo;
  chi[t] = (T)c;
  S[t] = (T)((lo * S_L[i] + chi_c[i] * B[i]) / c);
}

template <typename T>
__global__ void broadcast_kernel(int64_t n, int32_t nl, const double *__restrict__ v, T *__restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nl) return;
  out[t] = (T)v[t / nl];
}

__global__ void zero_u64_kernel(unsigned long long *p) { *p = 0ull; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One wavefront per site (grid-stride over sites), lanes over wavelengths.
template <typename T>
__global__ __launch_bounds__(256) void line_update_kernel(int64_t n, int32_t nl, int32_t R, const T *__restrict__ I,
                                                          const double *__restrict__ w,
                                                          const double *__restrict__ wlam,
                                                          const double *__restrict__ phi,
                                                          const double *__restrict__ B, double eps,
                                                          double *__restrict__ S_L, unsigned long long *dS_bits) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t nn = n * nl;
  double dmax = 0.0;
  for (int64_t i = wave; i < n; i += waves) {
    double acc = 0.0;
    for (int l = lane; l < nl; l += 64) {
      const int64_t q = i * nl + l;
      double j = 0.0;
      for (int32_t r = 0; r < R; ++r) j += w[r] * (double)I[(int64_t)r * nn + q];
      acc += wlam[l] * phi[q] * j;
    }
    const double jbar = wave_sum(acc);
    const double s_old = S_L[i];
    const double s_new = (1.0 - eps) * jbar + eps * B[i];
    const double d = fabs(s_new - s_old) / fabs(s_old);
    // NaN compares false: keep it so the host sees a non-finite change
    dmax = (d > dmax || d != d) ? d : dmax;
    if (lane == 0) S_L[i] = s_new;
  }
  // block maximum, then one atomic per block; non-negative doubles order like
  // their bit patterns and NaN sorts above +inf
  __shared__ double wmax[4];
  if (lane == 0) wmax[threadIdx.x >> 6] = dmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = wmax[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) m = (wmax[k] > m || wmax[k] != wmax[k]) ? wmax[k] : m;
    atomicMax(dS_bits, (unsigned long long)__double_as_longlong(m));
  }
}

inline unsigned nb(int64_t work, int bs) { return (unsigned)((work + bs - 1) / bs); }

}  // namespace

namespace vrt {

template <typename T>
void launch_nlte_assemble(hipStream_t s, int64_t n, int32_t nl, const double *phi, const double *chi_L,
                          const double *chi_c, const double *B, const double *S_L, T *chi, T *S) {
  if (n * nl == 0) return;
  hipLaunchKernelGGL(nlte_assemble_kernel<T>, dim3(nb(n * nl, 256)), dim3(256), 0, s, n, nl, phi, chi_L, chi_c, B,
                     S_L, chi, S);
  VRT_HIP(hipGetLastError());
}

template <typename T> void launch_broadcast(hipStream_t s, int64_t n, int32_t nl, const double *v, T *out) {
  if (n * nl == 0) return;
  hipLaunchKernelGGL(broadcast_kernel<T>, dim3(nb(n * nl, 256)), dim3(256), 0, s, n, nl, v, out);
  VRT_HIP(hipGetLastError());
}

void launch_zero_u64(hipStream_t s, unsigned long long *p) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, p);
  VRT_HIP(hipGetLastError());
}

template <typename T>
void launch_line_update(hipStream_t s, int64_t n, int32_t nl, int32_t R, const T *I, const double *w,
                        const double *wlam, const double *phi, const double *B, double eps, double *S_L,
                        unsigned long long *dS_bits) {
  if (n == 0) return;
  int64_t blocks = (n + 3) / 4;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(line_update_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, n, nl, R, I, w, wlam, phi, B,
                     eps, S_L, dS_bits);
  VRT_HIP(hipGetLastError());
}

template void launch_nlte_assemble<float>(hipStream_t, int64_t, int32_t, const double *, const double *,
                                          const double *, const double *, const double *, float *, float *);
template void launch_nlte_assemble<double>(hipStream_t, int64_t, int32_t, const double *, const double *,
                                           const double *, const double *, const double *, double *, double *);
template void launch_broadcast<float>(hipStream_t, int64_t, int32_t, const double *, float *);
template void launch_broadcast<double>(hipStream_t, int64_t, int32_t, const double *, double *);
template void launch_line_update<float>(hipStream_t, int64_t, int32_t, int32_t, const float *, const double *,
                                        const double *, const double *, const double *, double, double *,
                                        unsigned long long *);
template void launch_line_update<double>(hipStream_t, int64_t, int32_t, int32_t, const double *, const double *,
                                         const double *, const double *, const double *, double, double *,
                                         unsigned long long *);

}  // namespace vrt
