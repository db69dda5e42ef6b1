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
// only in wavelength and point; each wavefront covers 64/C consecutive points
// of one grid row (x direction) of one ray, with C lanes striding over
// wavelengths, V wavelengths (16 bytes) per lane when the rows allow it.
// Because the ray, the row and the plane geometry are the same for the whole
// wavefront, they are computed once per wavefront in scalar registers; only the
// point's x index and the wavelength differ between lanes.

#include "segment.h"
#include "vrt_internal.h"

namespace {

// Lane-vector of V elements (16-byte loads and stores when V > 1).
template <typename T, int V> struct RLane {
  typedef T type __attribute__((ext_vector_type(V)));
  static __device__ __forceinline__ type load(const T *p) { return *reinterpret_cast<const type *>(p); }
  static __device__ __forceinline__ void store(T *p, const type &v) { *reinterpret_cast<type *>(p) = v; }
};
template <typename T> struct RLane<T, 1> {
  typedef T type;
  static __device__ __forceinline__ type load(const T *p) { return *p; }
  static __device__ __forceinline__ void store(T *p, const type &v) { *p = v; }
};
template <typename T, int V> __device__ __forceinline__ T el(const typename RLane<T, V>::type &v, int k) {
  if constexpr (V == 1) return v;
  else return v[k];
}
template <typename T, int V> __device__ __forceinline__ void set_el(typename RLane<T, V>::type &v, int k, T x) {
  if constexpr (V == 1) v = x;
  else v[k] = x;
}

// The upwind point of every grid point of a plane is the point itself shifted
// by -ds (mx, my); on a uniform grid the cell offset and the bilinear weights
// are therefore the same for the whole plane: q / d = i + shift + t with an
// integer shift and 0 <= t < 1. The shift is reduced modulo np in double
// precision (exact for integers below 2^53); the two corrections catch the
// quotient's rounding.
__device__ __forceinline__ void plane_shift(double q_over_d, int32_t np, int32_t &shift, double &t) {
  const double fl = floor(q_over_d);
  t = q_over_d - fl;
  const double dn = (double)np;
  double m = fl - dn * floor(fl / dn);
  if (m < 0.0) m += dn;
  if (m >= dn) m -= dn;
  shift = (int32_t)m;  // in [0, np)
}

// Bilinear interpolation with a fixed order of operations, so that the row
// kernel and the tiled kernel round alike.
template <typename T>
__device__ __forceinline__ T bilin(T a00, T a10, T a01, T a11, T v00, T v10, T v01, T v11) {
#pragma clang fp contract(off)
  return vrt::seg_fma(a11, v11, vrt::seg_fma(a01, v01, vrt::seg_fma(a10, v10, a00 * v00)));
}

// C lanes per point, V consecutive wavelengths per lane (nl a multiple of V).
template <typename T, int C, int V>
__global__ __launch_bounds__(256) void regular_kernel(int32_t step, int32_t ray_begin, int32_t ray_count, int32_t nx,
                                                      int32_t ny, int32_t nz, double dx, double dy,
                                                      const double *__restrict__ z, const double *__restrict__ dirs,
                                                      int32_t nl, const T *__restrict__ chi, const T *__restrict__ S,
                                                      const T *__restrict__ Ibot, const T *__restrict__ Itop, T *I) {
  using L = RLane<T, V>;
  using VT = typename L::type;
  constexpr int SPW = 64 / C;
  const int lane = threadIdx.x & 63;
  // wavefront -> (ray, row j, first x of the wavefront), all wave-uniform
  const uint32_t wave = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  const uint32_t wpr = ((uint32_t)nx + SPW - 1) / SPW;
  const uint32_t row = wave / wpr;
  if (row >= (uint32_t)ray_count * (uint32_t)ny) return;
  const uint32_t rr = row / (uint32_t)ny;
  const int32_t j = (int32_t)(row - rr * (uint32_t)ny);
  const int32_t i = (int32_t)((wave - row * wpr) * SPW) + lane / C;
  if (i >= nx) return;
  const int l0 = (lane % C) * V;
  const int32_t r = ray_begin + (int32_t)rr;
  const int64_t plane = (int64_t)nx * ny;
  const int64_t p = (int64_t)j * nx + i;
  const double mx = dirs[3 * r + 0], my = dirs[3 * r + 1], mz = dirs[3 * r + 2];
  const bool up = mz > 0.0;
  const int32_t k = up ? step : nz - 1 - step;
  const int64_t n = plane * nz;
  T *Iray = I + (int64_t)r * n * nl;
  const int64_t me = ((int64_t)k * plane + p) * nl;
  if (step == 0) {
    for (int l = l0; l < nl; l += C * V) {
      VT v;
      if (up) v = L::load(Ibot + me + l);
      else if (Itop) v = L::load(Itop + me + l);
      else v = VT(T(0));
      L::store(Iray + me + l, v);
    }
    return;
  }
  const int32_t ku = up ? k - 1 : k + 1;
  const double ds = fabs(z[k] - z[ku]) / fabs(mz);
  int32_t sx, sy;
  double tx, ty;
  plane_shift(-ds * mx / dx, nx, sx, tx);
  plane_shift(-ds * my / dy, ny, sy, ty);
  int32_t ix0 = i + sx, iy0 = j + sy;
  if (ix0 >= nx) ix0 -= nx;
  if (iy0 >= ny) iy0 -= ny;
  const int32_t ix1 = ix0 + 1 == nx ? 0 : ix0 + 1, iy1 = iy0 + 1 == ny ? 0 : iy0 + 1;
  const T a00 = (T)((1.0 - tx) * (1.0 - ty)), a10 = (T)(tx * (1.0 - ty));
  const T a01 = (T)((1.0 - tx) * ty), a11 = (T)(tx * ty);
  const int64_t pu0 = (int64_t)ku * plane;
  const int64_t c00 = (pu0 + (int64_t)iy0 * nx + ix0) * nl, c10 = (pu0 + (int64_t)iy0 * nx + ix1) * nl;
  const int64_t c01 = (pu0 + (int64_t)iy1 * nx + ix0) * nl, c11 = (pu0 + (int64_t)iy1 * nx + ix1) * nl;
  const T h = (T)(0.5 * ds);
  for (int l = l0; l < nl; l += C * V) {
    const VT i00 = L::load(Iray + c00 + l), i10 = L::load(Iray + c10 + l);
    const VT i01 = L::load(Iray + c01 + l), i11 = L::load(Iray + c11 + l);
    const VT s00 = L::load(S + c00 + l), s10 = L::load(S + c10 + l);
    const VT s01 = L::load(S + c01 + l), s11 = L::load(S + c11 + l);
    const VT x00 = L::load(chi + c00 + l), x10 = L::load(chi + c10 + l);
    const VT x01 = L::load(chi + c01 + l), x11 = L::load(chi + c11 + l);
    const VT cm = L::load(chi + me + l), sm = L::load(S + me + l);
    VT out;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const T Iu = bilin<T>(a00, a10, a01, a11, el<T, V>(i00, e), el<T, V>(i10, e), el<T, V>(i01, e), el<T, V>(i11, e));
      const T Su = bilin<T>(a00, a10, a01, a11, el<T, V>(s00, e), el<T, V>(s10, e), el<T, V>(s01, e), el<T, V>(s11, e));
      const T cu = bilin<T>(a00, a10, a01, a11, el<T, V>(x00, e), el<T, V>(x10, e), el<T, V>(x01, e), el<T, V>(x11, e));
      set_el<T, V>(out, e, vrt::seg_line<T>((cu + el<T, V>(cm, e)) * h, Iu, Su, el<T, V>(sm, e)));
    }
    L::store(Iray + me + l, out);
  }
}

// LDS-tiled plane step (planes after the first). A workgroup owns an 8 x 8
// tile of grid points of one ray and a chunk of 4 lane-vectors (64 bytes) of
// their wavelengths. Because the upwind offset is the same for the whole
// plane, the upwind points of the tile form a 9 x 9 block of the previous
// plane; the workgroup stages chi, S and I of that block in LDS once (each
// upwind value is used by up to four points) and then updates every point
// from LDS, reading only its own chi and S from memory. Blocks are handed to
// the dies in contiguous ranges of tiles, so neighbouring tiles, which share
// the edge of their blocks, share a die's L2 (and the wavelength chunks of one
// tile are consecutive blocks). Same arithmetic as the row kernel.
constexpr int kTile = 8, kTileQ = 4;

template <typename T>
__global__ __launch_bounds__(256) void regular_tile_kernel(int32_t step, int32_t ray_begin, int32_t ray_count,
                                                           int32_t nx, int32_t ny, int32_t nz, double dx, double dy,
                                                           const double *__restrict__ z,
                                                           const double *__restrict__ dirs, int32_t nl,
                                                           const T *__restrict__ chi, const T *__restrict__ S, T *I,
                                                           int32_t xcd_chunks) {
  constexpr int V = 16 / (int)sizeof(T);
  using L = RLane<T, V>;
  using VT = typename L::type;
  constexpr int RX = kTile + 1, RP = RX * RX, Q = kTileQ;
  __shared__ VT reg[3][RP][Q];  // chi, S and I of the upwind block
  const int32_t tiles_x = (nx + kTile - 1) / kTile, tiles_y = (ny + kTile - 1) / kTile;
  const int64_t ntile = (int64_t)tiles_x * tiles_y;
  const int32_t nch = (nl + Q * V - 1) / (Q * V);
  // die-chunked block order (as in the Voronoi sweep)
  int64_t b = blockIdx.x;
  {
    const int64_t nb = gridDim.x, k = xcd_chunks;
    if (k > 1 && nb >= k) {
      const int64_t x = b % k, jj = b / k, per = nb / k, rem = nb % k;
      b = x * per + (x < rem ? x : rem) + jj;
    }
  }
  // wavelength chunks fastest: the chunks of one tile read the same rows
  const int32_t chunk = (int32_t)(b % nch);
  const int64_t rest = b / nch;
  const int64_t tile = rest % ntile;
  const int32_t rr = (int32_t)(rest / ntile);
  if (rr >= ray_count) return;  // uniform over the workgroup, before its barrier
  const int32_t r = ray_begin + rr;
  const int64_t plane = (int64_t)nx * ny;
  const double mx = dirs[3 * r + 0], my = dirs[3 * r + 1], mz = dirs[3 * r + 2];
  const bool up = mz > 0.0;
  const int32_t k = up ? step : nz - 1 - step;
  const int32_t ku = up ? k - 1 : k + 1;
  const int64_t n = plane * nz;
  T *Iray = I + (int64_t)r * n * nl;
  const double ds = fabs(z[k] - z[ku]) / fabs(mz);
  int32_t sx, sy;
  double tx, ty;
  plane_shift(-ds * mx / dx, nx, sx, tx);
  plane_shift(-ds * my / dy, ny, sy, ty);
  const int32_t x0 = (int32_t)(tile % tiles_x) * kTile, y0 = (int32_t)(tile / tiles_x) * kTile;
  const int32_t lc = chunk * Q * V;
  // stage the upwind block: point (a, c) of the block is grid point
  // (x0 + sx + a, y0 + sy + c) of plane ku, periodic in x and y
  const int64_t pu0 = (int64_t)ku * plane;
  for (int e = threadIdx.x; e < 3 * RP * Q; e += blockDim.x) {
    const int arr = e / (RP * Q), pq = e - arr * (RP * Q);
    const int p = pq / Q, q = pq - p * Q;
    const int a = p % RX, c = p / RX;
    int32_t gx = x0 + sx + a, gy = y0 + sy + c;
    while (gx >= nx) gx -= nx;
    while (gy >= ny) gy -= ny;
    const int32_t l = lc + q * V;
    VT v = VT(T(0));
    if (l < nl) {
      const int64_t off = (pu0 + (int64_t)gy * nx + gx) * nl + l;
      v = L::load((arr == 0 ? chi : arr == 1 ? S : Iray) + off);
    }
    reg[arr][p][q] = v;
  }
  __syncthreads();
  const int t = threadIdx.x;
  const int q = t % Q, pt = t / Q;
  const int px = pt % kTile, py = pt / kTile;
  const int32_t i = x0 + px, j = y0 + py, l = lc + q * V;
  if (i >= nx || j >= ny || l >= nl) return;
  const T a00 = (T)((1.0 - tx) * (1.0 - ty)), a10 = (T)(tx * (1.0 - ty));
  const T a01 = (T)((1.0 - tx) * ty), a11 = (T)(tx * ty);
  const T h = (T)(0.5 * ds);
  const int p00 = py * RX + px, p10 = p00 + 1, p01 = p00 + RX, p11 = p01 + 1;
  const int64_t me = ((int64_t)k * plane + (int64_t)j * nx + i) * nl + l;
  const VT cm = L::load(chi + me), sm = L::load(S + me);
  VT out;
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const T Iu = bilin<T>(a00, a10, a01, a11, el<T, V>(reg[2][p00][q], e), el<T, V>(reg[2][p10][q], e),
                          el<T, V>(reg[2][p01][q], e), el<T, V>(reg[2][p11][q], e));
    const T Su = bilin<T>(a00, a10, a01, a11, el<T, V>(reg[1][p00][q], e), el<T, V>(reg[1][p10][q], e),
                          el<T, V>(reg[1][p01][q], e), el<T, V>(reg[1][p11][q], e));
    const T cu = bilin<T>(a00, a10, a01, a11, el<T, V>(reg[0][p00][q], e), el<T, V>(reg[0][p10][q], e),
                          el<T, V>(reg[0][p01][q], e), el<T, V>(reg[0][p11][q], e));
    set_el<T, V>(out, e, vrt::seg_line<T>((cu + el<T, V>(cm, e)) * h, Iu, Su, el<T, V>(sm, e)));
  }
  L::store(Iray + me, out);
}

template <typename T, int C, int V>
void launch_rc(hipStream_t s, int32_t step, int32_t rb, int32_t rc, int32_t nx, int32_t ny, int32_t nz, double dx,
               double dy, const double *z, const double *dirs, int32_t nl, const T *chi, const T *S, const T *Ibot,
               const T *Itop, T *I) {
  constexpr int SPW = 64 / C;
  const int64_t waves = (int64_t)rc * ny * ((nx + SPW - 1) / SPW);
  const int64_t blocks = (waves + 3) / 4;
  if (waves >= (int64_t)1 << 31) throw vrt::Error(VRT_E_ARG, "regular grid too large for one plane launch");
  hipLaunchKernelGGL((regular_kernel<T, C, V>), dim3((unsigned)blocks), dim3(256), 0, s, step, rb, rc, nx, ny, nz, dx,
                     dy, z, dirs, nl, chi, S, Ibot, Itop, I);
}

template <typename T, int V>
void launch_rv(hipStream_t s, int32_t step, int32_t rb, int32_t rc, int32_t nx, int32_t ny, int32_t nz, double dx,
               double dy, const double *z, const double *dirs, int32_t nl, const T *chi, const T *S, const T *Ibot,
               const T *Itop, T *I) {
  switch (vrt::lanes_per_record(nl / V)) {
    case 64: launch_rc<T, 64, V>(s, step, rb, rc, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, Ibot, Itop, I); break;
    case 32: launch_rc<T, 32, V>(s, step, rb, rc, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, Ibot, Itop, I); break;
    case 16: launch_rc<T, 16, V>(s, step, rb, rc, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, Ibot, Itop, I); break;
    case 8: launch_rc<T, 8, V>(s, step, rb, rc, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, Ibot, Itop, I); break;
    case 4: launch_rc<T, 4, V>(s, step, rb, rc, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, Ibot, Itop, I); break;
    case 2: launch_rc<T, 2, V>(s, step, rb, rc, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, Ibot, Itop, I); break;
    default: launch_rc<T, 1, V>(s, step, rb, rc, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, Ibot, Itop, I); break;
  }
}

inline bool al16r(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

namespace vrt {

template <typename T>
void launch_regular(hipStream_t s, int32_t step, int32_t ray_begin, int32_t ray_count, int32_t nx, int32_t ny,
                    int32_t nz, double dx, double dy, const double *z, const double *dirs, int32_t nl, const T *chi,
                    const T *S, const T *Ibot, const T *Itop, T *I, bool tiled, int32_t xcd_chunks) {
  if (ray_count <= 0 || nx * ny == 0) return;
  constexpr int VW = 16 / sizeof(T);
  const bool aligned = al16r(chi) && al16r(S) && al16r(Ibot) && al16r(Itop) && al16r(I);
  if (tiled && step > 0 && aligned && nl % VW == 0) {
    const int64_t tiles = (int64_t)((nx + kTile - 1) / kTile) * ((ny + kTile - 1) / kTile);
    const int64_t blocks = tiles * ((nl + kTileQ * VW - 1) / (kTileQ * VW)) * ray_count;
    if (blocks >= (int64_t)1 << 31) throw Error(VRT_E_ARG, "regular grid too large for one plane launch");
    hipLaunchKernelGGL(regular_tile_kernel<T>, dim3((unsigned)blocks), dim3(kTile * kTile * kTileQ), 0, s, step,
                       ray_begin, ray_count, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, I, xcd_chunks);
    VRT_HIP(hipGetLastError());
    return;
  }
  if (aligned && nl % VW == 0)
    launch_rv<T, VW>(s, step, ray_begin, ray_count, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, Ibot, Itop, I);
  else
    launch_rv<T, 1>(s, step, ray_begin, ray_count, nx, ny, nz, dx, dy, z, dirs, nl, chi, S, Ibot, Itop, I);
  VRT_HIP(hipGetLastError());
}

template void launch_regular<float>(hipStream_t, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t, double, double,
                                    const double *, const double *, int32_t, const float *, const float *,
                                    const float *, const float *, float *, bool, int32_t);
template void launch_regular<double>(hipStream_t, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t, double, double,
                                     const double *, const double *, int32_t, const double *, const double *,
                                     const double *, const double *, double *, bool, int32_t);

}  // namespace vrt
