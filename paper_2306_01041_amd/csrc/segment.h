// Segment weights of the linear-source formal solution (Sect. 2.1 Eq. 2 with
// S linear along a segment of optical depth x, Sect. 2.5):
//   I = e^-x I_u + Psi_u(x) S_u + Psi_0(x) S_0,
//   Psi_0 = 1 - (1 - e^-x)/x,  Psi_u = (1 - e^-x)/x - e^-x.
// Below x = 1/2 both come from their power series
//   Psi_0 = sum_{n>=1} (-1)^(n+1) x^n/(n+1)!,  Psi_u = sum_{n>=1} (-1)^(n+1) n x^n/(n+1)!,
// which removes the 0/0 at x = 0 and the cancellation of the closed form at
// small x. The reverse sweep also needs the derivatives: dPsi_0/dx = Psi_u / x
// (whose series is the Psi_u series divided by x) and dPsi_u/dx = e^-x -
// dPsi_0/dx. Shared by the Voronoi, regular-grid and reverse sweeps.
#pragma once

#include <hip/hip_runtime.h>

namespace vrt {

template <typename T> struct Seg;

template <> struct Seg<float> {
  // ten terms: truncation below 1e-12 relative for x < 1/2
  static __device__ __forceinline__ void weights(float x, float &E, float &pu, float &p0) {
    float d0;
    weights(x, E, pu, p0, d0);
  }
  // also d0 = dPsi_0/dx = Psi_u / x (then dPsi_u/dx = e^-x - d0)
  static __device__ __forceinline__ void weights(float x, float &E, float &pu, float &p0, float &d0) {
    if (x < 0.5f) {
      // Psi_0 = sum_{n>=1} (-1)^(n+1) x^n/(n+1)!, Psi_u = sum (-1)^(n+1) n x^n/(n+1)!
      const float a = 1.0f / 39916800.0f;  // 1/11!
      float s0 = -a;
      s0 = s0 * x + 1.0f / 3628800.0f;
      s0 = s0 * x - 1.0f / 362880.0f;
      s0 = s0 * x + 1.0f / 40320.0f;
      s0 = s0 * x - 1.0f / 5040.0f;
      s0 = s0 * x + 1.0f / 720.0f;
      s0 = s0 * x - 1.0f / 120.0f;
      s0 = s0 * x + 1.0f / 24.0f;
      s0 = s0 * x - 1.0f / 6.0f;
      s0 = s0 * x + 0.5f;
      float su = -10.0f / 39916800.0f;
      su = su * x + 9.0f / 3628800.0f;
      su = su * x - 8.0f / 362880.0f;
      su = su * x + 7.0f / 40320.0f;
      su = su * x - 6.0f / 5040.0f;
      su = su * x + 5.0f / 720.0f;
      su = su * x - 4.0f / 120.0f;
      su = su * x + 3.0f / 24.0f;
      su = su * x - 2.0f / 6.0f;
      su = su * x + 0.5f;
      p0 = s0 * x;
      pu = su * x;
      d0 = su;
      E = expf(-x);
    } else {
      E = expf(-x);
      const float r = (1.0f - E) / x;
      p0 = 1.0f - r;
      pu = r - E;
      d0 = pu / x;
    }
  }
};

// 1/m! evaluated by the compiler
__host__ __device__ constexpr double inv_factorial(int m) {
  double f = 1.0;
  for (int i = 2; i <= m; ++i) f *= (double)i;
  return 1.0 / f;
}

template <> struct Seg<double> {
  // eighteen terms: truncation below 1e-21 relative for x < 1/2
  static __device__ __forceinline__ void weights(double x, double &E, double &pu, double &p0) {
    double d0;
    weights(x, E, pu, p0, d0);
  }
  static __device__ __forceinline__ void weights(double x, double &E, double &pu, double &p0, double &d0) {
    if (x < 0.5) {
      double s0 = 0.0, su = 0.0;
#pragma unroll
      for (int k = 18; k >= 1; --k) {
        const double c = ((k & 1) ? 1.0 : -1.0) * inv_factorial(k + 1);  // (-1)^(k+1)/(k+1)!
        s0 = s0 * x + c;
        su = su * x + (double)k * c;
      }
      p0 = s0 * x;
      pu = su * x;
      d0 = su;
      E = exp(-x);
    } else {
      E = exp(-x);
      const double r = -expm1(-x) / x;
      p0 = 1.0 - r;
      pu = r - E;
      d0 = pu / x;
    }
  }
};

}  // namespace vrt
