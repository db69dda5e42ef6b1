// Short characteristics on a regular grid (Sect. 2.6: the reference solver,
// with linear interpolation of the quantities at the upwind point).
//
// Plane by plane along each ray: the upwind point of grid point (i, j) in
// plane k is r - ds n in the adjacent plane k - sign(mu), with
// ds = |z_k - z_k'| / |mu|; I, S and chi there are interpolated bilinearly
// (periodic in x and y) and the same linear-source segment step as on the
// Voronoi grid is applied. Plane 0 (upward rays) takes I_bottom, the top plane
// (downward rays) I_top or zero.
//
// One launch handles one plane step of a contiguous block of rays. The
// bilinear weights are the same for every point of a plane, so lanes differ
// only in wavelength and point; each wavefront covers 64/C points of one ray
// with C lanes striding over wavelengths.

#include "segment.h"
#include "vrt_internal.h"

namespace {

__device__ __forceinline__ void periodic_cell(double q, double d, int32_t np, int32_t &i0, int32_t &i1, double &t) {
  const double f = q / d;
  const double fl = floor(f);
  t = f - fl;
  int64_t a = (int64_t)fl % np;
  if (a < 0) a += np;
  i0 = (int32_t)a;
  i1 = (int32_t)((a + 1) % np);
}

template <typename T, int C>
__global__ __launch_bounds__(256) void regular_kernel(int32_t step, int32_t ray_begin, int32_t ray_count, int32_t nx,
                                                      int32_t ny, int32_t nz, double dx, double dy,
                                                      const double *__restrict__ z, const double *__restrict__ dirs,
                                                      int32_t nl, const T *__restrict__ chi, const T *__restrict__ S,
                                                      const T *__restrict__ Ibot, const T *__restrict__ Itop, T *I) {
  constexpr int SPW = 64 / C;
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t plane = (int64_t)nx * ny;
  const int64_t item = wave * SPW + lane / C;
  const int l0 = lane % C;
  if (item >= plane * ray_count) return;
  const int32_t r = ray_begin + (int32_t)(item / plane);
  const int64_t p = item - (int64_t)(r - ray_begin) * plane;
  const int32_t i = (int32_t)(p % nx), j = (int32_t)(p / nx);
  const double mx = dirs[3 * r + 0], my = dirs[3 * r + 1], mz = dirs[3 * r + 2];
  const bool up = mz > 0.0;
  const int32_t k = up ? step : nz - 1 - step;
  const int64_t n = plane * nz;
  T *Iray = I + (int64_t)r * n * nl;
  const int64_t me = ((int64_t)k * plane + p) * nl;
  if (step == 0) {
    for (int l = l0; l < nl; l += C) {
      T v = T(0);
      if (up) v = Ibot[me + l];
      else if (Itop) v = Itop[me + l];
      Iray[me + l] = v;
    }
    return;
  }
  const int32_t ku = up ? k - 1 : k + 1;
  const double ds = fabs(z[k] - z[ku]) / fabs(mz);
  int32_t ix0, ix1, iy0, iy1;
  double tx, ty;
  periodic_cell((double)i * dx - ds * mx, dx, nx, ix0, ix1, tx);
  periodic_cell((double)j * dy - ds * my, dy, ny, iy0, iy1, ty);
  const T a00 = (T)((1.0 - tx) * (1.0 - ty)), a10 = (T)(tx * (1.0 - ty));
  const T a01 = (T)((1.0 - tx) * ty), a11 = (T)(tx * ty);
  const int64_t pu0 = (int64_t)ku * plane;
  const int64_t c00 = (pu0 + (int64_t)iy0 * nx + ix0) * nl, c10 = (pu0 + (int64_t)iy0 * nx + ix1) * nl;
  const int64_t c01 = (pu0 + (int64_t)iy1 * nx + ix0) * nl, c11 = (pu0 + (int64_t)iy1 * nx + ix1) * nl;
  const T h = (T)(0.5 * ds);
  for (int l = l0; l < nl; l += C) {
    const T Iu = a00 * Iray[c00 + l] + a10 * Iray[c10 + l] + a01 * Iray[c01 + l] + a11 * Iray[c11 + l];
    const T Su = a00 * S[c00 + l] + a10 * S[c10 + l] + a01 * S[c01 + l] + a11 * S[c11 + l];
    const T cu = a00 * chi[c00 + l] + a10 * chi[c10 + l] + a01 * chi[c01 + l] + a11 * chi[c11 + l];
    T E, pw, p0;
    vrt::Seg<T>::weights((cu + chi[me + l]) * h, E, pw, p0);
    Iray[me + l] = E * Iu + pw * Su + p0 * S[me + l];
  }
}

template <typename T, int C>
void launch_rc(hipStream_t s, int32_t step, int32_t rb, int32_t rc, int32_t nx, int32_t ny, int32_t nz, double dx,
               double dy, const double *z, const double *dirs, int32_t nl, const T *chi, const T *S, const T *Ibot,
               const T *Itop, T *I) {
  constexpr int SPW = 64 / C;
  const int64_t items = (int64_t)nx * ny * rc;
  const int64_t waves = (items + SPW - 1) / SPW;
  const int64_t blocks = (waves + 3) / 4;
  hipLaunchKernelGGL((regular_kernel<T, C>), dim3((unsigned)blocks), dim3(256), 0, s, step, rb, rc, nx, ny, nz, dx,
                     dy, z, dirs, nl, chi, S, Ibot, Itop, I);
}

}  // namespace

namespace vrt {

template <typename T>
void launch_regular(hipStream_t s, int32_t step, int32_t ray_begin, int32_t ray_count, int32_t nx, int32_t ny,
                    int32_t nz, double dx, double dy, const double *z, const double *dirs, int32_t nl, const T *chi,
                    const T *S, const T *Ibot, const T *Itop, T *I) {
  if (ray_count <= 0 || nx * ny == 0) return;
  if (nl >= 33) launch_rc<T, 64>(s, step, ray_begin, ray_count, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, Ibot, Itop, I);
  else if (nl >= 17) launch_rc<T, 32>(s, step, ray_begin, ray_count, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, Ibot, Itop, I);
  else if (nl >= 9) launch_rc<T, 16>(s, step, ray_begin, ray_count, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, Ibot, Itop, I);
  else if (nl >= 5) launch_rc<T, 8>(s, step, ray_begin, ray_count, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, Ibot, Itop, I);
  else if (nl >= 3) launch_rc<T, 4>(s, step, ray_begin, ray_count, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, Ibot, Itop, I);
  else if (nl == 2) launch_rc<T, 2>(s, step, ray_begin, ray_count, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, Ibot, Itop, I);
  else launch_rc<T, 1>(s, step, ray_begin, ray_count, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, Ibot, Itop, I);
  VRT_HIP(hipGetLastError());
}

template void launch_regular<float>(hipStream_t, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t, double, double,
                                    const double *, const double *, int32_t, const float *, const float *,
                                    const float *, const float *, float *);
template void launch_regular<double>(hipStream_t, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t, double, double,
                                     const double *, const double *, int32_t, const double *, const double *,
                                     const double *, const double *, double *);

}  // namespace vrt
