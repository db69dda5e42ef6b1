// Upwind selection on the GPU (Sect. 2.5, Eq. 5 and 6): for every ray and
// site, the two Delaunay lines closest in angle to the ray among the
// neighbours lying strictly upwind in height with a positive projection on
// the ray, and their weights w_j = v_j^r / (v_1^r + v_2^r).
//
// The ranking is integer output that must be reproducible bit for bit on any
// IEEE-754 machine, so the key of a line d (pointing from neighbour k into
// site i) is formed with plain +, -, *, / in a fixed order and no fused
// multiply-add: q = (n.d) |n.d| / |d|^2, which orders lines like the cosine
// v = n.d / |d|. Equal keys are broken by the smaller neighbour index, then by
// the earlier neighbour-list entry. Sites whose cell touches the upwind wall
// are boundary sites (no upwind lines). If no neighbour lies ahead of the ray,
// the z-upwind line with the largest key is used alone ("fallback").
//
// One thread per (ray, site); the neighbour list (about 15.5 entries) is read
// once per ray.

#include "vrt_internal.h"

namespace {

struct Line {
  int32_t k;
  int64_t e;
  double q, dot, len2;
};

__device__ __forceinline__ bool ranks_before(const Line &a, const Line &b) {
  if (a.q != b.q) return a.q > b.q;
  if (a.k != b.k) return a.k < b.k;
  return a.e < b.e;
}

__global__ __launch_bounds__(256) void select_kernel(
    int64_t n, int32_t R, const double *__restrict__ xyz, const int64_t *__restrict__ ptr,
    const int32_t *__restrict__ idx, const int8_t *__restrict__ shift, const uint8_t *__restrict__ wall,
    double Lx, double Ly, const double *__restrict__ dirs, double r_exp, int32_t *__restrict__ k1o,
    int32_t *__restrict__ k2o, double *__restrict__ w1o, double *__restrict__ ds1o, double *__restrict__ ds2o,
    unsigned long long *__restrict__ n_fallback, int32_t *__restrict__ bad_site) {
#pragma clang fp contract(off)
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)R * n) return;
  const int32_t r = (int32_t)(t / n);
  const int64_t i = t - (int64_t)r * n;
  const double rx = dirs[3 * r + 0], ry = dirs[3 * r + 1], rz = dirs[3 * r + 2];
  const bool up = rz > 0.0;
  int32_t out_k1 = -1, out_k2 = -1;
  double out_w1 = 1.0, out_d1 = 0.0, out_d2 = 0.0;
  if (!(wall[i] & (up ? 1 : 2))) {
    const double xi = xyz[3 * i + 0], yi = xyz[3 * i + 1], zi = xyz[3 * i + 2];
    Line b1{-1, -1, 0.0, 0.0, 1.0}, b2 = b1, fb = b1;
    int nc = 0, nz = 0;
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
      const int32_t k = idx[e];
      const double dxs = (double)shift[2 * e + 0] * Lx;
      const double dys = (double)shift[2 * e + 1] * Ly;
      const double dx = (xi - xyz[3 * k + 0]) - dxs;
      const double dy = (yi - xyz[3 * k + 1]) - dys;
      const double dz = zi - xyz[3 * k + 2];
      const bool zup = up ? (dz > 0.0) : (dz < 0.0);
      if (!zup) continue;
      Line c;
      c.k = k;
      c.e = e;
      const double px = rx * dx;
      const double py = ry * dy;
      const double pz = rz * dz;
      c.dot = (px + py) + pz;
      const double sx = dx * dx;
      const double sy = dy * dy;
      const double sz = dz * dz;
      c.len2 = (sx + sy) + sz;
      c.q = (c.dot * fabs(c.dot)) / c.len2;
      if (nz == 0 || ranks_before(c, fb)) fb = c;
      ++nz;
      if (c.dot > 0.0) {
        if (nc == 0) {
          b1 = c;
        } else if (ranks_before(c, b1)) {
          b2 = b1;
          b1 = c;
        } else if (nc == 1 || ranks_before(c, b2)) {
          b2 = c;
        }
        ++nc;
      }
    }
    if (nc >= 2) {
      const double v1 = b1.dot / sqrt(b1.len2);
      const double v2 = b2.dot / sqrt(b2.len2);
      const double p1 = pow(v1, r_exp), p2 = pow(v2, r_exp);
      out_k1 = b1.k;
      out_k2 = b2.k;
      out_w1 = p1 / (p1 + p2);
      out_d1 = sqrt(b1.len2);
      out_d2 = sqrt(b2.len2);
    } else if (nc == 1) {
      out_k1 = b1.k;
      out_d1 = sqrt(b1.len2);
    } else if (nz > 0) {
      out_k1 = fb.k;
      out_d1 = sqrt(fb.len2);
      atomicAdd(&n_fallback[r], 1ull);
    } else {
      atomicMin(bad_site, (int32_t)i);
    }
  }
  k1o[t] = out_k1;
  k2o[t] = out_k2;
  w1o[t] = out_w1;
  ds1o[t] = out_d1;
  ds2o[t] = out_d2;
}

}  // namespace

namespace vrt {

void launch_select(hipStream_t s, int64_t n, int32_t R, const double *xyz, const int64_t *ptr,
                   const int32_t *idx, const int8_t *shift, const uint8_t *wall, double Lx, double Ly,
                   const double *dirs, double r_exp, int32_t *k1, int32_t *k2, double *w1, double *ds1,
                   double *ds2, unsigned long long *n_fallback, int32_t *bad_site) {
  const int64_t total = (int64_t)R * n;
  if (total == 0) return;
  const int64_t blocks = (total + 255) / 256;
  hipLaunchKernelGGL(select_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n, R, xyz, ptr, idx, shift, wall,
                     Lx, Ly, dirs, r_exp, k1, k2, w1, ds1, ds2, n_fallback, bad_site);
  VRT_HIP(hipGetLastError());
}

}  // namespace vrt
