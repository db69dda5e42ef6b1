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

// Vector of V elements (16-byte stores when V > 1).
template <typename T, int V> struct SVec {
  typedef T type __attribute__((ext_vector_type(V)));
};
template <typename T> struct SVec<T, 1> {
  typedef T type;
};

// C lanes per site (a power of two), 64/C sites per wavefront, V consecutive
// wavelengths per lane (nl a multiple of V): the site's temperature, density
// and opacity are loaded once per lane group, each lane evaluates the Planck
// function at its V wavelengths, and a wavefront writes whole rows. Rows of
// site i start at i cs (cs >= nl, a multiple of V).
template <typename T, int C, int V>
__global__ __launch_bounds__(256) void lte_kernel(int64_t n, int32_t nl, int64_t cs, const double *__restrict__ lam,
                                                  double kappa0, const double *__restrict__ Tk,
                                                  const double *__restrict__ rho, T *__restrict__ chi,
                                                  T *__restrict__ S) {
  using VT = typename SVec<T, V>::type;
  constexpr int SPW = 64 / C;
  const int lane = threadIdx.x & 63;
  const int64_t i = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * SPW + lane / C;
  if (i >= n) return;
  const double Ti = Tk[i], ri = rho[i];
  const double T3 = Ti * Ti * Ti;
  const T c = (T)(kappa0 * (ri * ri) * (T3 * T3 * T3));
  T *crow = chi + i * cs, *srow = S + i * cs;
  for (int32_t l = (lane % C) * V; l < nl; l += C * V) {
    VT cv, sv;
    if constexpr (V == 1) {
      cv = c;
      sv = (T)planck_kw_nm(lam[l], Ti);
    } else {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        cv[e] = c;
        sv[e] = (T)planck_kw_nm(lam[l + e], Ti);
      }
    }
    *reinterpret_cast<VT *>(crow + l) = cv;
    *reinterpret_cast<VT *>(srow + l) = sv;
  }
}

template <typename T, int C, int V>
void launch_lc(hipStream_t s, int64_t n, int32_t nl, int64_t cs, const double *lam, double kappa0, const double *T_,
               const double *rho, T *chi, T *S) {
  constexpr int SPW = 64 / C;
  const int64_t blocks = (n + 4 * SPW - 1) / (4 * SPW);
  hipLaunchKernelGGL((lte_kernel<T, C, V>), dim3((unsigned)blocks), dim3(256), 0, s, n, nl, cs, lam, kappa0, T_, rho,
                     chi, S);
}

template <typename T, int V>
void launch_lv(hipStream_t s, int64_t n, int32_t nl, int64_t cs, const double *lam, double kappa0, const double *T_,
               const double *rho, T *chi, T *S) {
  switch (vrt::lanes_per_record(nl / V)) {
    case 64: launch_lc<T, 64, V>(s, n, nl, cs, lam, kappa0, T_, rho, chi, S); break;
    case 32: launch_lc<T, 32, V>(s, n, nl, cs, lam, kappa0, T_, rho, chi, S); break;
    case 16: launch_lc<T, 16, V>(s, n, nl, cs, lam, kappa0, T_, rho, chi, S); break;
    case 8: launch_lc<T, 8, V>(s, n, nl, cs, lam, kappa0, T_, rho, chi, S); break;
    case 4: launch_lc<T, 4, V>(s, n, nl, cs, lam, kappa0, T_, rho, chi, S); break;
    case 2: launch_lc<T, 2, V>(s, n, nl, cs, lam, kappa0, T_, rho, chi, S); break;
    default: launch_lc<T, 1, V>(s, n, nl, cs, lam, kappa0, T_, rho, chi, S); break;
  }
}

inline bool al16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

namespace vrt {

template <typename T>
void launch_lte(hipStream_t s, int64_t n, int32_t nl, int64_t cs, const double *lam, double kappa0, const double *T_,
                const double *rho, T *chi, T *S) {
  if (n == 0 || nl == 0) return;
  constexpr int VW = 16 / sizeof(T);
  if (nl % VW == 0 && cs % VW == 0 && al16(chi) && al16(S))
    launch_lv<T, VW>(s, n, nl, cs, lam, kappa0, T_, rho, chi, S);
  else
    launch_lv<T, 1>(s, n, nl, cs, lam, kappa0, T_, rho, chi, S);
  VRT_HIP(hipGetLastError());
}

template void launch_lte<float>(hipStream_t, int64_t, int32_t, int64_t, const double *, double, const double *,
                                const double *, float *, float *);
template void launch_lte<double>(hipStream_t, int64_t, int32_t, int64_t, const double *, double, const double *,
                                 const double *, double *, double *);

}  // namespace vrt
