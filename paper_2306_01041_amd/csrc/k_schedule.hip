// Per-ray level schedules of the upwind dependency graph and the packing of
// sweep records (rays start at the upwind boundary and advance site by site,
// Sect. 2.5). A site's level is 0 at the boundary and otherwise one more than
// the largest level among the (at most two) sites it reads from; all sites of
// one level can be updated in parallel once the earlier levels are done.
//
// Levels are found by monotone relaxation: start every site at level 0 and
// repeatedly set level(i) = 1 + max(level(k1), level(k2)). Values only grow
// and are bounded by the longest path, so a pass without change is the fixed
// point; concurrent reads of a neighbour being updated only delay that pass.
// The order (level, site index) is a stable counting sort: each thread owns a
// tile of consecutive visiting positions, counts levels inside it, an
// exclusive scan over (level, tile) gives every tile's first slot per level,
// and the tiles scatter their sites in visiting order. Visiting the sites in
// index order gives the (level, index) order; visiting them through another
// permutation (e.g. a space-filling curve) orders each level by it instead.

#include "vrt_internal.h"

namespace {

__global__ void level_fill_kernel(int64_t total, int32_t *__restrict__ level) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < total) level[t] = 0;
}

__global__ __launch_bounds__(256) void level_relax_kernel(int64_t n, int32_t R, const int32_t *__restrict__ k1,
                                                          const int32_t *__restrict__ k2, int32_t *level,
                                                          int32_t *changed) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)R * n) return;
  const int64_t base = (t / n) * n;
  const int32_t a = k1[t];
  if (a < 0) return;  // boundary sites stay at level 0
  const int32_t b = k2[t];
  int32_t v = __hip_atomic_load(&level[base + a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (b >= 0) {
    const int32_t vb = __hip_atomic_load(&level[base + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v = vb > v ? vb : v;
  }
  v += 1;
  if (v != level[t]) {
    __hip_atomic_store(&level[t], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *changed = 1;
  }
}

// Levels shared by a group of rays (peer[r][0..P) lists the rays that share
// ray r's levels, -1 padded): a site's level is the same for every ray of the
// group and exceeds the level of every site that any of them reads from, the
// longest path in the union of their dependency graphs. Starting from zero (or
// from any lower bound) the relaxation only raises levels, as above.
__global__ __launch_bounds__(256) void level_share_kernel(int64_t n, int32_t R, int32_t P,
                                                          const int32_t *__restrict__ peer,
                                                          const int32_t *__restrict__ k1,
                                                          const int32_t *__restrict__ k2, int32_t *level,
                                                          int32_t *changed) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)R * n) return;
  const int32_t r = (int32_t)(t / n);
  const int64_t i = t - (int64_t)r * n;
  int32_t v = __hip_atomic_load(&level[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int32_t p = 0; p < P; ++p) {
    const int32_t q = peer[(int64_t)r * P + p];
    if (q < 0) break;
    const int64_t bq = (int64_t)q * n;
    const int32_t lq = __hip_atomic_load(&level[bq + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v = lq > v ? lq : v;
    const int32_t a = k1[bq + i];
    if (a < 0) continue;
    const int32_t va = __hip_atomic_load(&level[bq + a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
    v = va > v ? va : v;
    const int32_t b = k2[bq + i];
    if (b >= 0) {
      const int32_t vb = __hip_atomic_load(&level[bq + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
      v = vb > v ? vb : v;
    }
  }
  if (v != level[t]) {
    __hip_atomic_store(&level[t], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *changed = 1;
  }
}

__global__ void level_max_kernel(int64_t total, const int32_t *__restrict__ level, int32_t *out_max) {
  int32_t m = 0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x)
    m = level[t] > m ? level[t] : m;
  atomicMax(out_max, m);
}

// cnt layout: [R][Lmax][ntiles]
__global__ void level_count_kernel(int64_t n, int32_t R, int32_t Lmax, int64_t tile, int64_t ntiles,
                                   const int32_t *__restrict__ level, int32_t *__restrict__ cnt,
                                   const int32_t *__restrict__ visit) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)R * ntiles) return;
  const int32_t r = (int32_t)(t / ntiles);
  const int64_t tl = t - (int64_t)r * ntiles;
  const int64_t i0 = tl * tile, i1 = (i0 + tile < n) ? i0 + tile : n;
  int32_t *c = cnt + (int64_t)r * Lmax * ntiles + tl;
  for (int64_t j = i0; j < i1; ++j) {
    const int64_t i = visit ? visit[j] : j;
    c[(int64_t)level[(int64_t)r * n + i] * ntiles] += 1;
  }
}

// one thread per (ray, level): exclusive scan over tiles, level total out
__global__ void level_scan_kernel(int32_t R, int32_t Lmax, int64_t ntiles, int32_t *__restrict__ cnt,
                                  int64_t *__restrict__ totals) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)R * Lmax) return;
  int32_t *c = cnt + t * ntiles;
  int64_t run = 0;
  for (int64_t j = 0; j < ntiles; ++j) {
    const int32_t v = c[j];
    c[j] = (int32_t)run;
    run += v;
  }
  totals[t] = run;
}

// one thread per ray: level_ptr [R][Lmax + 1] and the number of levels
__global__ void level_ptr_kernel(int32_t R, int32_t Lmax, const int64_t *__restrict__ totals,
                                 int32_t *__restrict__ level_ptr, int32_t *__restrict__ n_levels) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  int64_t p = 0;
  int32_t last = 0;
  for (int32_t l = 0; l < Lmax; ++l) {
    level_ptr[(int64_t)r * (Lmax + 1) + l] = (int32_t)p;
    const int64_t c = totals[(int64_t)r * Lmax + l];
    if (c > 0) last = l;
    p += c;
  }
  level_ptr[(int64_t)r * (Lmax + 1) + Lmax] = (int32_t)p;
  n_levels[r] = last + 1;
}

__global__ void level_scatter_kernel(int64_t n, int32_t R, int32_t Lmax, int64_t tile, int64_t ntiles,
                                     const int32_t *__restrict__ level, const int32_t *__restrict__ level_ptr,
                                     int32_t *__restrict__ cnt, int32_t *__restrict__ order,
                                     const int32_t *__restrict__ visit) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)R * ntiles) return;
  const int32_t r = (int32_t)(t / ntiles);
  const int64_t tl = t - (int64_t)r * ntiles;
  const int64_t i0 = tl * tile, i1 = (i0 + tile < n) ? i0 + tile : n;
  int32_t *c = cnt + (int64_t)r * Lmax * ntiles + tl;
  const int32_t *lp = level_ptr + (int64_t)r * (Lmax + 1);
  for (int64_t j = i0; j < i1; ++j) {
    const int64_t i = visit ? visit[j] : j;
    const int32_t l = level[(int64_t)r * n + i];
    const int64_t slot = (int64_t)lp[l] + c[(int64_t)l * ntiles];
    c[(int64_t)l * ntiles] += 1;
    order[(int64_t)r * n + slot] = (int32_t)i;
  }
}

// one thread per (ray, position in the ray's order)
__global__ __launch_bounds__(256) void pack_kernel(int64_t n, int32_t R, int32_t Lmax,
                                                   const int32_t *__restrict__ order,
                                                   const int32_t *__restrict__ level,
                                                   const int32_t *__restrict__ level_ptr,
                                                   const int64_t *__restrict__ seg_off, const int32_t *__restrict__ k1,
                                                   const int32_t *__restrict__ k2, const double *__restrict__ w1,
                                                   const double *__restrict__ ds1, const double *__restrict__ ds2,
                                                   const double *__restrict__ dirs, int4 *__restrict__ ri,
                                                   vrt::RecF32 *__restrict__ rf32, vrt::RecF64 *__restrict__ rf64) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)R * n) return;
  const int32_t r = (int32_t)(t / n);
  const int64_t p = t - (int64_t)r * n;
  const int32_t site = order[t];
  const int64_t rs = (int64_t)r * n + site;
  const int32_t l = level[rs];
  const int64_t g = seg_off[(int64_t)l * R + r] + (p - level_ptr[(int64_t)r * (Lmax + 1) + l]);
  const int up = dirs[3 * r + 2] > 0.0 ? 1 : 0;
  ri[g] = make_int4(site, k1[rs], k2[rs], 2 * r + up);
  rf32[g] = vrt::RecF32{(float)w1[rs], (float)ds1[rs], (float)ds2[rs], 0.0f};
  rf64[g] = vrt::RecF64{w1[rs], ds1[rs], ds2[rs], 0.0};
}

inline unsigned nblocks(int64_t total, int bs) { return vrt::grid_blocks(total, bs); }

}  // namespace

namespace vrt {

void launch_level_fill(hipStream_t s, int64_t total, int32_t *level) {
  if (total == 0) return;
  hipLaunchKernelGGL(level_fill_kernel, dim3(nblocks(total, 256)), dim3(256), 0, s, total, level);
  VRT_HIP(hipGetLastError());
}

void launch_level_relax(hipStream_t s, int64_t n, int32_t R, const int32_t *k1, const int32_t *k2,
                        int32_t *level, int32_t *changed, const int32_t *peer, int32_t P) {
  const int64_t total = (int64_t)R * n;
  if (total == 0) return;
  if (peer)
    hipLaunchKernelGGL(level_share_kernel, dim3(nblocks(total, 256)), dim3(256), 0, s, n, R, P, peer, k1, k2, level,
                       changed);
  else
    hipLaunchKernelGGL(level_relax_kernel, dim3(nblocks(total, 256)), dim3(256), 0, s, n, R, k1, k2, level, changed);
  VRT_HIP(hipGetLastError());
}

void launch_level_max(hipStream_t s, int64_t total, const int32_t *level, int32_t *out_max) {
  if (total == 0) return;
  unsigned b = nblocks(total, 256);
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(level_max_kernel, dim3(b), dim3(256), 0, s, total, level, out_max);
  VRT_HIP(hipGetLastError());
}

void launch_level_count(hipStream_t s, int64_t n, int32_t R, int32_t Lmax, int64_t tile, const int32_t *level,
                        int32_t *cnt, const int32_t *visit) {
  const int64_t ntiles = (n + tile - 1) / tile;
  const int64_t total = (int64_t)R * ntiles;
  if (total == 0) return;
  hipLaunchKernelGGL(level_count_kernel, dim3(nblocks(total, 64)), dim3(64), 0, s, n, R, Lmax, tile, ntiles,
                     level, cnt, visit);
  VRT_HIP(hipGetLastError());
}

void launch_level_scan(hipStream_t s, int32_t R, int32_t Lmax, int64_t ntiles, int32_t *cnt, int64_t *totals) {
  const int64_t total = (int64_t)R * Lmax;
  if (total == 0) return;
  hipLaunchKernelGGL(level_scan_kernel, dim3(nblocks(total, 64)), dim3(64), 0, s, R, Lmax, ntiles, cnt, totals);
  VRT_HIP(hipGetLastError());
}

void launch_level_ptr(hipStream_t s, int32_t R, int32_t Lmax, const int64_t *totals, int32_t *level_ptr,
                      int32_t *n_levels) {
  if (R == 0) return;
  hipLaunchKernelGGL(level_ptr_kernel, dim3(nblocks(R, 64)), dim3(64), 0, s, R, Lmax, totals, level_ptr, n_levels);
  VRT_HIP(hipGetLastError());
}

void launch_level_scatter(hipStream_t s, int64_t n, int32_t R, int32_t Lmax, int64_t tile, const int32_t *level,
                          const int32_t *level_ptr, int32_t *cnt, int32_t *order, const int32_t *visit) {
  const int64_t ntiles = (n + tile - 1) / tile;
  const int64_t total = (int64_t)R * ntiles;
  if (total == 0) return;
  hipLaunchKernelGGL(level_scatter_kernel, dim3(nblocks(total, 64)), dim3(64), 0, s, n, R, Lmax, tile, ntiles,
                     level, level_ptr, cnt, order, visit);
  VRT_HIP(hipGetLastError());
}

void launch_pack(hipStream_t s, int64_t n, int32_t R, int32_t Lmax, const int32_t *order, const int32_t *level,
                 const int32_t *level_ptr, const int64_t *seg_off, const int32_t *k1, const int32_t *k2,
                 const double *w1, const double *ds1, const double *ds2, const double *dirs, int4 *ri,
                 RecF32 *rf32, RecF64 *rf64) {
  const int64_t total = (int64_t)R * n;
  if (total == 0) return;
  hipLaunchKernelGGL(pack_kernel, dim3(nblocks(total, 256)), dim3(256), 0, s, n, R, Lmax, order, level, level_ptr,
                     seg_off, k1, k2, w1, ds1, ds2, dirs, ri, rf32, rf64);
  VRT_HIP(hipGetLastError());
}

}  // namespace vrt
