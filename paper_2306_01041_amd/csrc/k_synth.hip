// Final synthesis on the original regular grid (Sect. 2.5, closing
// paragraph; Sect. 3.2): quantities converged on the Voronoi grid are carried
// back to the regular points by inverse-distance weights of the two nearest
// sites, and the emergent intensity at mu = 1 is a long-characteristics
// solution up each vertical column.
//
// Nearest sites. The site nearest to a point p is found by a greedy walk over
// the Voronoi neighbour lists: from a start site, move to the neighbour with
// the smallest key (d^2, site index) while that key is smaller than the
// current one. A Voronoi cell is the intersection of the half-spaces cut by
// its face neighbours, so a site that no neighbour beats holds p in its cell
// (the walk stops exactly at the nearest site; periodic images are handled by
// the minimum-image distance, and the box walls clip every cell the same
// way). The second-nearest site shares a face with the nearest one: shrinking
// the empty ball about p that passes through the second site, towards that
// site, until it touches the first gives an empty ball through both, whose
// centre lies inside the (convex) box. So the scan of the nearest site's list
// that confirms the walk's end also yields the second site. Points are
// processed coarse to fine: the points of a coarse lattice (points x sites at
// most 2^24) by brute force over all sites, then lattices of half the stride
// down to every point, each new point walking from the nearest site of its
// parent on the previous lattice, so walks are a few steps long. Distances use
// the same operations in the same order as their definition and no fused
// multiply-add, so the chosen sites are reproducible on any IEEE-754 machine.
//
// Columns. One thread per (column, wavelength); consecutive threads take
// consecutive wavelengths and then columns, so each horizontal plane of a
// [point][lambda] array is read as one contiguous stream. Every thread walks
// its column from the bottom plane to the top with the linear-source step.

#include "segment.h"
#include "vrt_internal.h"

namespace {

// d reduced into [-L/2, L/2] by one period: the host guarantees that points
// lie in [0, L) and the box starts within half a period of 0, so |d| < 3L/2
// and one shift suffices (the same result as repeated shifts)
__device__ __forceinline__ double wrap_period(double d, int periodic, double L) {
  const double h = 0.5 * L;
  const double up = d < -h ? d + L : d;
  return periodic ? (d > h ? d - L : up) : d;
}

__device__ __forceinline__ double point_dist2(double px, double py, double pz, double sx, double sy, double sz,
                                              int periodic, double Lx, double Ly) {
#pragma clang fp contract(off)
  const double dx = wrap_period(px - sx, periodic, Lx);
  const double dy = wrap_period(py - sy, periodic, Ly);
  const double dz = pz - sz;
  return dx * dx + dy * dy + dz * dz;
}

__device__ __forceinline__ double site_dist2(double px, double py, double pz, const double *__restrict__ xyz,
                                             int32_t s, int periodic, double Lx, double Ly) {
  return point_dist2(px, py, pz, xyz[3 * (int64_t)s + 0], xyz[3 * (int64_t)s + 1], xyz[3 * (int64_t)s + 2],
                     periodic, Lx, Ly);
}

__device__ __forceinline__ bool key_less(double da, int32_t ia, double db, int32_t ib) {
  return da < db || (da == db && ia < ib);
}

// entries of a neighbour list, or sites of a brute-force scan, loaded together
constexpr int kScan = 8;

// insert (site s, key d) into the two smallest keys so far (s < 0: nothing)
__device__ __forceinline__ void top2_insert(int32_t s, double d, int32_t &b1, double &e1, int32_t &b2, double &e2) {
  if (s < 0) return;
  if (b1 < 0 || key_less(d, s, e1, b1)) {
    b2 = b1;
    e2 = e1;
    b1 = s;
    e1 = d;
  } else if (b2 < 0 || key_less(d, s, e2, b2)) {
    b2 = s;
    e2 = d;
  }
}

// Weight of the nearer site, u_k = d_k^-power normalised: w1 = a_2/(a_1 + a_2)
// with a_k = (d2_k)^(power/2), 1 when the point is a site; a lone site is its
// own second neighbour.
__device__ __forceinline__ void store_pair(int64_t p, int32_t i1, double e1, int32_t i2, double e2, double power,
                                           int32_t *__restrict__ idx, double *__restrict__ w1,
                                           double *__restrict__ d2) {
  double w = 1.0;
  if (i1 < 0) {
    i2 = -1;
    w = __builtin_nan("");
  } else if (i2 < 0) {
    i2 = i1;
    e2 = e1;
  } else {
    const double a1 = pow(e1, 0.5 * power), a2 = pow(e2, 0.5 * power);
    if (a1 + a2 > 0.0) w = a2 / (a1 + a2);
  }
  idx[2 * p + 0] = i1;
  idx[2 * p + 1] = i2;
  w1[p] = w;
  if (d2) {
    d2[2 * p + 0] = e1;
    d2[2 * p + 1] = e2;
  }
}

__global__ __launch_bounds__(256) void idw_level_kernel(int32_t nx, int32_t ny, int32_t nz, double dx, double dy,
                                                        const double *__restrict__ z, int32_t stride,
                                                        int32_t parent, int64_t n, const double *__restrict__ xyz,
                                                        const int64_t *__restrict__ ptr,
                                                        const int32_t *__restrict__ nbr, int periodic, double Lx,
                                                        double Ly, double power, int32_t *__restrict__ idx,
                                                        double *__restrict__ w1, double *__restrict__ d2,
                                                        int32_t *__restrict__ bad) {
  const int64_t cx = (nx + stride - 1) / stride, cy = (ny + stride - 1) / stride, cz = (nz + stride - 1) / stride;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cx * cy * cz) return;
  const int32_t i = (int32_t)(t % cx) * stride;
  const int32_t j = (int32_t)((t / cx) % cy) * stride;
  const int32_t k = (int32_t)(t / (cx * cy)) * stride;
  // points on the parent lattice were done by an earlier launch
  if (parent > 0 && i % parent == 0 && j % parent == 0 && k % parent == 0) return;
  const int64_t p = ((int64_t)k * ny + j) * nx + i;
  int32_t cur = 0;
  if (parent > 0) {
    const int64_t q = ((int64_t)(k / parent * parent) * ny + j / parent * parent) * nx + i / parent * parent;
    const int32_t s = idx[2 * q];
    if (s >= 0 && s < n) cur = s;
  }
  const double px = (double)i * dx, py = (double)j * dy, pz = z[k];
  double dc = site_dist2(px, py, pz, xyz, cur, periodic, Lx, Ly);
  int32_t i1 = -1, i2 = -1;
  double e1 = 0.0, e2 = 0.0;
  // the key falls at every move, so there are at most n - 1 moves
  for (int64_t it = 0; it < n; ++it) {
    int32_t b = -1;
    double db = 0.0;
    // the list is read kScan entries at a time, all indices and then all
    // coordinates of a batch in flight together
    const int64_t e_end = ptr[cur + 1];
    for (int64_t e0 = ptr[cur]; e0 < e_end; e0 += kScan) {
      int32_t sn[kScan];
      double sx[kScan], sy[kScan], sz[kScan];
#pragma unroll
      for (int u = 0; u < kScan; ++u) sn[u] = e0 + u < e_end ? nbr[e0 + u] : cur;
#pragma unroll
      for (int u = 0; u < kScan; ++u) {
        sx[u] = xyz[3 * (int64_t)sn[u] + 0];
        sy[u] = xyz[3 * (int64_t)sn[u] + 1];
        sz[u] = xyz[3 * (int64_t)sn[u] + 2];
      }
#pragma unroll
      for (int u = 0; u < kScan; ++u) {
        if (sn[u] == cur) continue;  // past the list's end, or a periodic image of the site itself
        const double d = point_dist2(px, py, pz, sx[u], sy[u], sz[u], periodic, Lx, Ly);
        if (b < 0 || key_less(d, sn[u], db, b)) {
          b = sn[u];
          db = d;
        }
      }
    }
    if (b >= 0 && key_less(db, b, dc, cur)) {
      cur = b;
      dc = db;
      continue;
    }
    i1 = cur;
    e1 = dc;
    i2 = b;
    e2 = db;
    break;
  }
  if (i1 < 0) *bad = 1;  // the walk did not settle: the neighbour lists are not a Voronoi diagram
  store_pair(p, i1, e1, i2, e2, power, idx, w1, d2);
}

// Two nearest sites of the points on one lattice by brute force, in two
// passes. First every workgroup takes kBrutePts points and one chunk of
// kBruteChunk sites: each thread reads a strided share of the chunk's sites
// once and keeps, for every one of the points, the two smallest keys; a tree
// merge in LDS per point leaves the chunk's two. Then one thread per point
// merges its chunks.
constexpr int64_t kBruteChunk = 8192;
constexpr int kBrutePts = 8;

__global__ __launch_bounds__(256) void idw_brute_partial_kernel(int32_t nx, int32_t ny, double dx, double dy,
                                                                const double *__restrict__ z, int32_t stride,
                                                                int64_t n_pts, int64_t n, int64_t n_chunks,
                                                                const double *__restrict__ xyz, int periodic,
                                                                double Lx, double Ly, int32_t *__restrict__ pb,
                                                                double *__restrict__ pe) {
  __shared__ double se1[256], se2[256];
  __shared__ int32_t sb1[256], sb2[256];
  const int64_t cx = (nx + stride - 1) / stride, cy = (ny + stride - 1) / stride;
  const int64_t blk = blockIdx.x;
  const int64_t g = blk / n_chunks, c = blk - g * n_chunks;
  double px[kBrutePts], py[kBrutePts], pz[kBrutePts];
  int32_t b1[kBrutePts], b2[kBrutePts];
  double e1[kBrutePts], e2[kBrutePts];
#pragma unroll
  for (int u = 0; u < kBrutePts; ++u) {
    // points past the lattice repeat its last point (their results are not stored)
    const int64_t q = g * kBrutePts + u < n_pts ? g * kBrutePts + u : n_pts - 1;
    px[u] = (double)((int32_t)(q % cx) * stride) * dx;
    py[u] = (double)((int32_t)((q / cx) % cy) * stride) * dy;
    pz[u] = z[(q / (cx * cy)) * stride];
    b1[u] = b2[u] = -1;
    e1[u] = e2[u] = 0.0;
  }
  const int64_t end = (c + 1) * kBruteChunk < n ? (c + 1) * kBruteChunk : n;
  // kScan sites per thread in flight at a time
  for (int64_t s0 = c * kBruteChunk + threadIdx.x; s0 < end; s0 += kScan * blockDim.x) {
    double sx[kScan], sy[kScan], sz[kScan];
#pragma unroll
    for (int v = 0; v < kScan; ++v) {
      const int64_t s = s0 + v * blockDim.x < end ? s0 + v * blockDim.x : s0;
      sx[v] = xyz[3 * s + 0];
      sy[v] = xyz[3 * s + 1];
      sz[v] = xyz[3 * s + 2];
    }
#pragma unroll
    for (int v = 0; v < kScan; ++v) {
      const int64_t s = s0 + v * blockDim.x;
      if (s >= end) break;
#pragma unroll
      for (int u = 0; u < kBrutePts; ++u) {
        const double d = point_dist2(px[u], py[u], pz[u], sx[v], sy[v], sz[v], periodic, Lx, Ly);
        if (b2[u] < 0 || d <= e2[u]) top2_insert((int32_t)s, d, b1[u], e1[u], b2[u], e2[u]);
      }
    }
  }
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < kBrutePts; ++u) {
    sb1[tid] = b1[u];
    se1[tid] = e1[u];
    sb2[tid] = b2[u];
    se2[tid] = e2[u];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) {
        int32_t a1 = sb1[tid], a2 = sb2[tid];
        double f1 = se1[tid], f2 = se2[tid];
        top2_insert(sb1[tid + h], se1[tid + h], a1, f1, a2, f2);
        top2_insert(sb2[tid + h], se2[tid + h], a1, f1, a2, f2);
        sb1[tid] = a1;
        se1[tid] = f1;
        sb2[tid] = a2;
        se2[tid] = f2;
      }
      __syncthreads();
    }
    const int64_t q = g * kBrutePts + u;
    if (tid == 0 && q < n_pts) {
      const int64_t r = 2 * (q * n_chunks + c);
      pb[r] = sb1[0];
      pb[r + 1] = sb2[0];
      pe[r] = se1[0];
      pe[r + 1] = se2[0];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void idw_brute_merge_kernel(int32_t nx, int32_t ny, int32_t nz, int32_t stride,
                                                              int64_t n_chunks, const int32_t *__restrict__ pb,
                                                              const double *__restrict__ pe, double power,
                                                              int32_t *__restrict__ idx, double *__restrict__ w1,
                                                              double *__restrict__ d2) {
  const int64_t cx = (nx + stride - 1) / stride, cy = (ny + stride - 1) / stride, cz = (nz + stride - 1) / stride;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= cx * cy * cz) return;
  int32_t b1 = -1, b2 = -1;
  double e1 = 0.0, e2 = 0.0;
  for (int64_t c = 0; c < n_chunks; ++c) {
    const int64_t r = 2 * (q * n_chunks + c);
    top2_insert(pb[r], pe[r], b1, e1, b2, e2);
    top2_insert(pb[r + 1], pe[r + 1], b1, e1, b2, e2);
  }
  const int32_t i = (int32_t)(q % cx) * stride;
  const int32_t j = (int32_t)((q / cx) % cy) * stride;
  const int32_t k = (int32_t)(q / (cx * cy)) * stride;
  store_pair(((int64_t)k * ny + j) * nx + i, b1, e1, b2, e2, power, idx, w1, d2);
}

__global__ __launch_bounds__(256) void idw_apply_kernel(int64_t m, int32_t nc, int64_t n_src,
                                                        const int32_t *__restrict__ idx, const double *__restrict__ w1,
                                                        const double *__restrict__ src, double *__restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * nc) return;
  const int64_t p = t / nc;
  const int32_t c = (int32_t)(t - p * nc);
  const int32_t a = idx[2 * p], b = idx[2 * p + 1];
  if (a < 0 || a >= n_src || b < 0 || b >= n_src) {
    dst[t] = __builtin_nan("");
    return;
  }
  const double w = w1[p];
  dst[t] = w * src[(int64_t)a * nc + c] + (1.0 - w) * src[(int64_t)b * nc + c];
}

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

// Per regular point: (chi_line, chi_cont, chi_cont (B - S_line), S_line), with
// S_line interpolated from the two nearest sites, formed in double precision
// and stored in the precision of the column pass. With chi = chi_cont +
// chi_line phi, the source (chi_line phi S_line + chi_cont B) / chi equals
// S_line + chi_cont (B - S_line) / chi, which costs one fused multiply-add and
// one quotient per wavelength.
template <typename T>
__global__ __launch_bounds__(256) void line_pack_kernel(int64_t m, int64_t n_src, const int32_t *__restrict__ idx,
                                                        const double *__restrict__ w1,
                                                        const double *__restrict__ S_site,
                                                        const double *__restrict__ chi_L,
                                                        const double *__restrict__ chi_c,
                                                        const double *__restrict__ B,
                                                        typename Vec4<T>::type *__restrict__ pack) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  const int32_t a = idx[2 * p], b = idx[2 * p + 1];
  double SL = __builtin_nan("");
  if (a >= 0 && a < n_src && b >= 0 && b < n_src) {
    const double w = w1[p];
    SL = w * S_site[a] + (1.0 - w) * S_site[b];
  }
  typename Vec4<T>::type v;
  v.x = (T)chi_L[p];
  v.y = (T)chi_c[p];
  v.z = (T)(chi_c[p] * (B[p] - SL));
  v.w = (T)SL;
  pack[p] = v;
}

// Quotient a / b: IEEE division in double precision; in single precision the
// hardware reciprocal (about 1 ulp) times a, which is what the column pass can
// afford per (point, wavelength, plane).
__device__ __forceinline__ double quot(double a, double b) { return a / b; }
__device__ __forceinline__ float quot(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// One linear-source step up a column, I <- e^-x I + Psi_u S_u + Psi_0 S_0.
// Double precision uses the shared segment weights in that form. Single
// precision uses the equivalent I <- S_u + e^-x (I - S_u) + Psi_0 (S_0 - S_u)
// (Psi_u = 1 - e^-x - Psi_0), which needs only e^-x and Psi_0 and keeps the
// rounding proportional to the differences; it evaluates both forms of Psi_0
// and selects, because the lanes of one wavefront hold different wavelengths,
// so optically thin and thick segments sit side by side and a branch would run
// both sides anyway: the series sum_{n=1..5} (-1)^(n+1) x^n/(n+1)! below
// x = 1/10 (the first omitted term is below 1e-8 of Psi_0 there) and
// 1 - (1 - e^-x)/x above, with e^-x from the hardware base-2 exponential.
template <typename T> struct ColumnStep {
  static __device__ __forceinline__ T advance(T I, T x, T Su, T S0) {
    T E, pu, p0;
    vrt::Seg<T>::weights(x, E, pu, p0);
    return E * I + pu * Su + p0 * S0;
  }
};
template <> struct ColumnStep<float> {
  static __device__ __forceinline__ float advance(float I, float x, float Su, float S0) {
    const float E = __builtin_amdgcn_exp2f(-x * 1.44269504088896341f);
    float s = 1.0f / 720.0f;
    s = s * x - 1.0f / 120.0f;
    s = s * x + 1.0f / 24.0f;
    s = s * x - 1.0f / 6.0f;
    s = s * x + 0.5f;
    const float closed = 1.0f - (1.0f - E) * __builtin_amdgcn_rcpf(x);
    const float p0 = x < 0.1f ? s * x : closed;
    return Su + E * (I - Su) + p0 * (S0 - Su);
  }
};

// Opacity and source of one (point, wavelength).
template <typename T> struct LineSource {
  const T *phi;
  const typename Vec4<T>::type *pack;
  __device__ __forceinline__ void at(int64_t p, int64_t pl, T &chi, T &S) const {
    const typename Vec4<T>::type v = pack[p];
    chi = v.y + v.x * phi[pl];
    S = v.w + quot(v.z, chi);
  }
};

template <typename T> struct PlainSource {
  const T *chi, *S;
  __device__ __forceinline__ void at(int64_t, int64_t pl, T &c, T &s) const {
    c = chi[pl];
    s = S[pl];
  }
};

// I_bottom defaults: the line synthesis enters with B of the bottom point, the
// plain solve with the bottom point's source function (thermalised).
template <typename T> __device__ __forceinline__ T default_bottom(const LineSource<T> &, const double *B, int64_t c, T) {
  return (T)B[c];
}
template <typename T> __device__ __forceinline__ T default_bottom(const PlainSource<T> &, const double *, int64_t, T S0) {
  return S0;
}

template <typename T, class Src>
__global__ __launch_bounds__(256) void vertical_kernel(int64_t ncol, int32_t nz, int32_t nl,
                                                       const double *__restrict__ z, Src src,
                                                       const double *__restrict__ B, const T *__restrict__ Ib,
                                                       T *__restrict__ out) {
  const int64_t plane = ncol * nl;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= plane) return;
  const int64_t c = t / nl;
  T chi0, S0;
  src.at(c, t, chi0, S0);
  T I = Ib ? Ib[t] : default_bottom(src, B, c, S0);
  constexpr int U = sizeof(T) == 4 ? 8 : 2;  // planes whose inputs are loaded before they are integrated
  int32_t k = 1;
  for (; k + U <= nz; k += U) {
    T chi1[U], S1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) src.at((int64_t)(k + u) * ncol + c, (int64_t)(k + u) * plane + t, chi1[u], S1[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T x = (chi0 + chi1[u]) * (T)(0.5 * (z[k + u] - z[k + u - 1]));
      I = ColumnStep<T>::advance(I, x, S0, S1[u]);
      chi0 = chi1[u];
      S0 = S1[u];
    }
  }
  for (; k < nz; ++k) {
    T chi1, S1;
    src.at((int64_t)k * ncol + c, (int64_t)k * plane + t, chi1, S1);
    const T x = (chi0 + chi1) * (T)(0.5 * (z[k] - z[k - 1]));
    I = ColumnStep<T>::advance(I, x, S0, S1);
    chi0 = chi1;
    S0 = S1;
  }
  out[t] = I;
}

inline unsigned blocks_for(int64_t count, int threads = 256) { return vrt::grid_blocks(count, threads); }

}  // namespace

namespace vrt {

void launch_idw_level(hipStream_t s, int32_t nx, int32_t ny, int32_t nz, double dx, double dy, const double *z,
                      int32_t stride, int32_t parent, int64_t n, const double *xyz, const int64_t *ptr,
                      const int32_t *nbr, bool periodic, double Lx, double Ly, double power, int32_t *idx,
                      double *w1, double *d2, int32_t *bad) {
  const int64_t cnt = (int64_t)((nx + stride - 1) / stride) * ((ny + stride - 1) / stride) *
                      ((nz + stride - 1) / stride);
  if (cnt == 0) return;
  idw_level_kernel<<<blocks_for(cnt), 256, 0, s>>>(nx, ny, nz, dx, dy, z, stride, parent, n, xyz, ptr, nbr,
                                                   periodic ? 1 : 0, Lx, Ly, power, idx, w1, d2, bad);
  VRT_HIP(hipGetLastError());
}

int64_t idw_brute_scratch_pairs(int32_t nx, int32_t ny, int32_t nz, int32_t stride, int64_t n) {
  const int64_t cnt = (int64_t)((nx + stride - 1) / stride) * ((ny + stride - 1) / stride) *
                      ((nz + stride - 1) / stride);
  return cnt * ((n + kBruteChunk - 1) / kBruteChunk);
}

void launch_idw_brute(hipStream_t s, int32_t nx, int32_t ny, int32_t nz, double dx, double dy, const double *z,
                      int32_t stride, int64_t n, const double *xyz, bool periodic, double Lx, double Ly, double power,
                      int32_t *idx, double *w1, double *d2, int32_t *pb, double *pe) {
  const int64_t cnt = (int64_t)((nx + stride - 1) / stride) * ((ny + stride - 1) / stride) *
                      ((nz + stride - 1) / stride);
  const int64_t n_chunks = (n + kBruteChunk - 1) / kBruteChunk;
  if (cnt == 0 || n_chunks == 0) return;
  const int64_t groups = (cnt + kBrutePts - 1) / kBrutePts;
  idw_brute_partial_kernel<<<(unsigned)(groups * n_chunks), 256, 0, s>>>(nx, ny, dx, dy, z, stride, cnt, n, n_chunks,
                                                                          xyz, periodic ? 1 : 0, Lx, Ly, pb, pe);
  VRT_HIP(hipGetLastError());
  idw_brute_merge_kernel<<<blocks_for(cnt), 256, 0, s>>>(nx, ny, nz, stride, n_chunks, pb, pe, power, idx, w1, d2);
  VRT_HIP(hipGetLastError());
}

void launch_idw_apply(hipStream_t s, int64_t m, int32_t nc, int64_t n_src, const int32_t *idx, const double *w1,
                      const double *src, double *dst) {
  if (m * nc == 0) return;
  idw_apply_kernel<<<blocks_for(m * nc), 256, 0, s>>>(m, nc, n_src, idx, w1, src, dst);
  VRT_HIP(hipGetLastError());
}

template <typename T>
void launch_line_pack(hipStream_t s, int64_t m, int64_t n_src, const int32_t *idx, const double *w1,
                      const double *S_site, const double *chi_L, const double *chi_c, const double *B, void *pack) {
  if (m == 0) return;
  line_pack_kernel<T><<<blocks_for(m), 256, 0, s>>>(m, n_src, idx, w1, S_site, chi_L, chi_c, B,
                                                    static_cast<typename Vec4<T>::type *>(pack));
  VRT_HIP(hipGetLastError());
}

template <typename T>
void launch_vertical_line(hipStream_t s, int64_t ncol, int32_t nz, int32_t nl, const double *z, const T *phi,
                          const void *pack, const double *B, const T *Ib, T *out) {
  if (ncol * nl == 0) return;
  LineSource<T> src{phi, static_cast<const typename Vec4<T>::type *>(pack)};
  vertical_kernel<T, LineSource<T>><<<blocks_for(ncol * nl), 256, 0, s>>>(ncol, nz, nl, z, src, B, Ib, out);
  VRT_HIP(hipGetLastError());
}

template <typename T>
void launch_vertical_plain(hipStream_t s, int64_t ncol, int32_t nz, int32_t nl, const double *z, const T *chi,
                           const T *S, const T *Ib, T *out) {
  if (ncol * nl == 0) return;
  PlainSource<T> src{chi, S};
  vertical_kernel<T, PlainSource<T>><<<blocks_for(ncol * nl), 256, 0, s>>>(ncol, nz, nl, z, src, nullptr, Ib, out);
  VRT_HIP(hipGetLastError());
}

template void launch_line_pack<float>(hipStream_t, int64_t, int64_t, const int32_t *, const double *, const double *,
                                      const double *, const double *, const double *, void *);
template void launch_line_pack<double>(hipStream_t, int64_t, int64_t, const int32_t *, const double *, const double *,
                                       const double *, const double *, const double *, void *);
template void launch_vertical_line<float>(hipStream_t, int64_t, int32_t, int32_t, const double *, const float *,
                                          const void *, const double *, const float *, float *);
template void launch_vertical_line<double>(hipStream_t, int64_t, int32_t, int32_t, const double *, const double *,
                                           const void *, const double *, const double *, double *);
template void launch_vertical_plain<float>(hipStream_t, int64_t, int32_t, int32_t, const double *, const float *,
                                           const float *, const float *, float *);
template void launch_vertical_plain<double>(hipStream_t, int64_t, int32_t, int32_t, const double *, const double *,
                                            const double *, const double *, double *);

}  // namespace vrt
