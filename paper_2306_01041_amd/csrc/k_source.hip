// Opacity and source assembly for the grey LTE continuum (Sect. 2.1 with the
// source function equal to the Planck function): chi = kappa0 rho^2 T^9, the
// same at every wavelength (a mass absorption coefficient kappa0 rho T^9 times
// the density), and S = B_lambda(T) in kW m^-2 nm^-1 sr^-1. Evaluated in
// double precision and stored in the sweep precision.

#include "vrt_internal.h"

namespace {

// SI 2019 exact values
constexpr double kPlanckH = 6.62607015e-34;   // J s
constexpr double kLightC = 299792458.0;       // m s^-1
constexpr double kBoltzmannK = 1.380649e-23;  // J K^-1

__device__ __forceinline__ double planck_kw_nm(double lam, double T) {
  const double hc = kPlanckH * kLightC;
  const double u = hc / (lam * (kBoltzmannK * T));
  const double l2 = lam * lam;
  const double l5 = l2 * l2 * lam;
  // W m^-2 m^-1 sr^-1 -> kW m^-2 nm^-1 sr^-1
  return (2.0 * hc * kLightC) / l5 / expm1(u) * 1.0e-12;
}

template <typename T>
__global__ __launch_bounds__(256) void lte_kernel(int64_t n, int32_t nl, const double *__restrict__ lam, double kappa0,
                                                  const double *__restrict__ Tk, const double *__restrict__ rho,
                                                  T *__restrict__ chi, T *__restrict__ S) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nl) return;
  const int64_t i = t / nl;
  const int32_t l = (int32_t)(t - i * nl);
  const double Ti = Tk[i], ri = rho[i];
  const double T3 = Ti * Ti * Ti;
  chi[t] = (T)(kappa0 * (ri * ri) * (T3 * T3 * T3));
  S[t] = (T)planck_kw_nm(lam[l], Ti);
}

}  // namespace

namespace vrt {

template <typename T>
void launch_lte(hipStream_t s, int64_t n, int32_t nl, const double *lam, double kappa0, const double *T_,
                const double *rho, T *chi, T *S) {
  const int64_t work = n * nl;
  if (work == 0) return;
  hipLaunchKernelGGL(lte_kernel<T>, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, n, nl, lam, kappa0, T_,
                     rho, chi, S);
  VRT_HIP(hipGetLastError());
}

template void launch_lte<float>(hipStream_t, int64_t, int32_t, const double *, double, const double *,
                                const double *, float *, float *);
template void launch_lte<double>(hipStream_t, int64_t, int32_t, const double *, double, const double *,
                                 const double *, double *, double *);

}  // namespace vrt
