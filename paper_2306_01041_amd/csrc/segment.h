// Segment weights of the linear-source formal solution (Sect. 2.1 Eq. 2 with
// S linear along a segment of optical depth x, Sect. 2.5):
//   I = e^-x I_u + Psi_u(x) S_u + Psi_0(x) S_0,
//   Psi_0 = 1 - (1 - e^-x)/x,  Psi_u = (1 - e^-x)/x - e^-x.
// Below x = 1/2 both come from their power series
//   Psi_0 = sum_{n>=1} (-1)^(n+1) x^n/(n+1)!,  Psi_u = sum_{n>=1} (-1)^(n+1) n x^n/(n+1)!,
// which removes the 0/0 at x = 0 and the cancellation of the closed form at
// small x (single precision forms Psi_u as x times the series of r - Psi_0/x,
// r = (1 - e^-x)/x, which is the same series). The reverse sweep also needs
// the derivatives: dPsi_0/dx = Psi_u / x (whose series is the Psi_u series
// divided by x) and dPsi_u/dx = e^-x - dPsi_0/dx. Shared by the Voronoi, regular-grid and reverse sweeps.
#pragma once

#include <hip/hip_runtime.h>

namespace vrt {

template <typename T> struct Seg;

template <> struct Seg<float> {
  static __device__ __forceinline__ void weights(float x, float &E, float &pu, float &p0) {
    float d0;
    weights(x, E, pu, p0, d0);
  }
  // Branchless: both forms are evaluated and the lane selects one, because the
  // lanes of a wavefront hold different wavelengths and sites and would
  // otherwise run both sides of a branch one after the other. With
  // r = (1 - e^-x)/x, Psi_0 = 1 - r and Psi_u = r - e^-x:
  //  * x >= 1/2: e^-x from the hardware base-2 exponential of -x log2(e)
  //    (relative error below 1e-6 for x < 10, where e^-x still matters) and
  //    r = (1 - e^-x) times the hardware reciprocal of x;
  //  * x < 1/2: Psi_0 = x P(x) and Psi_u = x (R(x) - P(x)) from the power
  //    series P = sum_{n>=1} (-1)^(n+1) x^(n-1)/(n+1)! (seven terms) and
  //    R = r = sum_{n>=0} (-1)^n x^n/(n+1)! (eight terms), truncated below
  //    1e-8 relative, so that Psi_0 and Psi_u keep their relative accuracy as
  //    x -> 0 (the closed form loses it to the cancellation in 1 - e^-x).
  // Worst relative error of Psi_0 and Psi_u over all x: 5e-7 and 8.4e-7 (at
  // x just above 1/2, from the rounding of e^-x).
  // Also d0 = dPsi_0/dx = Psi_u/x (then dPsi_u/dx = e^-x - d0).
  static __device__ __forceinline__ void weights(float x, float &E, float &pu, float &p0, float &d0) {
#pragma clang fp contract(off)
    E = __builtin_amdgcn_exp2f(x * -1.44269504088896341f);
    const float inv = __builtin_amdgcn_rcpf(x);
    const float rc = (1.0f - E) * inv;
    const float p0c = 1.0f - rc, puc = rc - E;
    float P = 1.0f / 40320.0f;  // P = 1/2 - x/6 + x^2/24 - ... + x^6/8!
    P = __builtin_fmaf(P, x, -1.0f / 5040.0f);
    P = __builtin_fmaf(P, x, 1.0f / 720.0f);
    P = __builtin_fmaf(P, x, -1.0f / 120.0f);
    P = __builtin_fmaf(P, x, 1.0f / 24.0f);
    P = __builtin_fmaf(P, x, -1.0f / 6.0f);
    P = __builtin_fmaf(P, x, 0.5f);
    float R = -1.0f / 40320.0f;  // R = 1 - x/2 + x^2/6 - ... - x^7/8!
    R = __builtin_fmaf(R, x, 1.0f / 5040.0f);
    R = __builtin_fmaf(R, x, -1.0f / 720.0f);
    R = __builtin_fmaf(R, x, 1.0f / 120.0f);
    R = __builtin_fmaf(R, x, -1.0f / 24.0f);
    R = __builtin_fmaf(R, x, 1.0f / 6.0f);
    R = __builtin_fmaf(R, x, -0.5f);
    R = __builtin_fmaf(R, x, 1.0f);
    const float Q = R - P;  // Psi_u / x
    const bool s = x < 0.5f;
    p0 = s ? x * P : p0c;
    pu = s ? x * Q : puc;
    d0 = s ? Q : puc * inv;
  }
};

// 1/m! evaluated by the compiler
__host__ __device__ constexpr double inv_factorial(int m) {
  double f = 1.0;
  for (int i = 2; i <= m; ++i) f *= (double)i;
  return 1.0 / f;
}

template <> struct Seg<double> {
  static __device__ __forceinline__ void weights(double x, double &E, double &pu, double &p0) {
    double d0;
    weights(x, E, pu, p0, d0);
  }
  // One exponential for both forms. Below x = 1/2 the forms of the single
  // precision path with longer series: Psi_0 = x P(x) and Psi_u = x (R(x) - P(x)),
  // R = sum_{n=0..16} (-1)^n x^n/(n+1)! (= (1 - e^-x)/x) and
  // P = sum_{n=1..16} (-1)^(n+1) x^(n-1)/(n+1)! (= (1 - R)/x), whose
  // coefficients are R's shifted by one with the sign changed; the first term
  // left out is below 1e-19 relative. From x = 1/2 up, 1 - e^-x >= 0.39
  // carries no cancellation, so r = (1 - e^-x)/x keeps double precision.
  static __device__ __forceinline__ void weights(double x, double &E, double &pu, double &p0, double &d0) {
    E = exp(-x);
    double R = inv_factorial(17);  // (-1)^16/17!
    double P = -inv_factorial(17);  // (-1)^17/17!, the x^15 term of P
#pragma unroll
    for (int n = 15; n >= 0; --n) {
      const double b = ((n & 1) ? -1.0 : 1.0) * inv_factorial(n + 1);  // (-1)^n/(n+1)!
      R = R * x + b;
      if (n >= 1) P = P * x - b;  // the x^(n-1) term of P is -(x^n term of R)
    }
    const double Q = R - P;  // Psi_u / x
    if (x < 0.5) {
      p0 = x * P;
      pu = x * Q;
      d0 = Q;
    } else {
      const double r = (1.0 - E) / x;
      p0 = 1.0 - r;
      pu = r - E;
      d0 = pu / x;
    }
  }
};

// single-rounding multiply-add of either precision
__device__ __forceinline__ float seg_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double seg_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One line of the segment update (Eq. 2 with S linear along the line):
// I = e^-x I_u + Psi_u S_u + Psi_0 S_0, rounded as
// fma(e^-x, I_u, fma(Psi_u, S_u, Psi_0 S_0)). Every sweep forms its lines and
// their Eq. 5 weighting with these two functions, with contraction off, so
// that launch modes and lane layouts that share a record give the same bits.
template <typename T> __device__ __forceinline__ T seg_line(T x, T Iu, T Su, T S0) {
#pragma clang fp contract(off)
  T E, pu, p0;
  Seg<T>::weights(x, E, pu, p0);
  return seg_fma(E, Iu, seg_fma(pu, Su, p0 * S0));
}

// Eq. 5 with two lines: w1 a + w2 b (w2 = 1 - w1), rounded as fma(w1, a, w2 b)
template <typename T> __device__ __forceinline__ T seg_mix(T w1, T w2, T a, T b) {
#pragma clang fp contract(off)
  return seg_fma(w1, a, w2 * b);
}

}  // namespace vrt
