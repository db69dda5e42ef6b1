// Formal-solution sweep on a Voronoi grid (Sect. 2.1 Eq. 2; Sect. 2.5 Eq. 5),
// the angle quadrature of J (Sect. 2.1 Eq. 4) and the emergent-intensity
// gather.
//
// One launch updates a contiguous range of sweep records: every site of one
// level of one ray (plain execution) or one level of every ray (batched). A
// wavefront of 64 lanes covers 64/C records with C lanes each, the lanes of a
// record striding over wavelengths, so every read and write of a
// [site][lambda] row is a contiguous, coalesced access; wavelengths are
// independent, so no lane ever waits for another.
//
// For each upwind line j (site k_j, length ds_j) the segment optical depth is
// the trapezoid x = (chi_k + chi_i) ds / 2 and, with S linear along the line,
//   I_j = e^-x I_k + Psi_u(x) S_k + Psi_0(x) S_i,
//   Psi_0 = 1 - (1 - e^-x)/x,  Psi_u = (1 - e^-x)/x - e^-x;
// below x = 1/2 both ratios come from their Taylor series (no 0/0 at x = 0, no
// cancellation). The site's intensity is w1 I_1 + (1 - w1) I_2 (Eq. 5).

#include "segment.h"
#include "vrt_internal.h"

namespace {

// Lane-vector of V elements (16-byte loads and stores when V > 1).
template <typename T, int V> struct Lane {
  typedef T type __attribute__((ext_vector_type(V)));
  static __device__ __forceinline__ type load(const T *p) { return *reinterpret_cast<const type *>(p); }
  static __device__ __forceinline__ void store(T *p, const type &v) { *reinterpret_cast<type *>(p) = v; }
  static __device__ __forceinline__ T get(const type &v, int k) { return v[k]; }
  static __device__ __forceinline__ void set(type &v, int k, T x) { v[k] = x; }
};
template <typename T> struct Lane<T, 1> {
  typedef T type;
  static __device__ __forceinline__ type load(const T *p) { return *p; }
  static __device__ __forceinline__ void store(T *p, const type &v) { *p = v; }
  static __device__ __forceinline__ T get(const type &v, int) { return v; }
  static __device__ __forceinline__ void set(type &v, int, T x) { v = x; }
};

// Workgroups are handed to the accelerator dies (XCDs) round-robin. With
// k > 1 chunks, block b is renumbered so that die (b mod k) works on the
// (b mod k)-th contiguous chunk of the launch's records: records that are
// neighbours in the (spatially sorted) record order share a die and its L2.
__device__ __forceinline__ int64_t chunked_block(int32_t k) {
  const int64_t b = blockIdx.x, nb = gridDim.x;
  if (k <= 1 || nb < k) return b;
  const int64_t x = b % k, j = b / k, per = nb / k, rem = nb % k;
  return x * per + (x < rem ? x : rem) + j;
}

// Ray affinity: each ray is assigned to one die for the whole sweep, so the
// rows a level writes are read by the next level through the same die's L2.
// The launch of one step passes that step's table xtab[die][k] = {first
// record, running record count} over the k < xk segments of the die's rays;
// block b works for die b mod 8. Returns the record of this lane, or -1.
__device__ __forceinline__ int64_t affinity_record(const int64_t *__restrict__ xtab, int32_t xk, int spw, int lane,
                                                   int c) {
  const int x = blockIdx.x & (vrt::kDies - 1);
  const int64_t j = ((int64_t)(blockIdx.x / vrt::kDies) * (blockDim.x >> 6) + (threadIdx.x >> 6)) * spw + lane / c;
  const int64_t *t = xtab + (int64_t)x * xk * 2;
  int64_t prev = 0;
  for (int32_t k = 0; k < xk; ++k) {
    const int64_t cum = t[2 * k + 1];
    if (j < cum) return t[2 * k] + (j - prev);
    prev = cum;
  }
  return -1;
}

// C lanes per record, V consecutive wavelengths per lane (nl and cs are
// multiples of V). The input rows of site i (chi, S and the boundary
// intensities) start at i cs (cs >= nl); intensity rows are nl apart.
template <typename T, int C, int V>
__device__ __forceinline__ void sweep_body(const int4 *__restrict__ ri,
                                           const typename vrt::RecOf<T>::type *__restrict__ rf, int64_t rec_begin,
                                           int64_t rec_count, int32_t nl, int64_t cs, int64_t n,
                                           const T *__restrict__ chi, const T *__restrict__ S,
                                           const T *__restrict__ Ibot,
                                           const T *__restrict__ Itop, T *I, int32_t xcd_chunks, int32_t ray0,
                                           const int64_t *__restrict__ xtab, int32_t xk) {
  using L = Lane<T, V>;
  using VT = typename L::type;
  constexpr int SPW = 64 / C;
  const int lane = threadIdx.x & 63;
  const int l0 = (lane % C) * V;
  int64_t rec;
  if (xtab) {
    rec = affinity_record(xtab, xk, SPW, lane, C);
    if (rec < 0) return;
  } else {
    const int64_t wave = chunked_block(xcd_chunks) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t r = wave * SPW + lane / C;
    if (r >= rec_count) return;
    rec = rec_begin + r;
  }
  const int4 q = ri[rec];
  const int32_t site = q.x, k1 = q.y, k2 = q.z;
  const int32_t ray = q.w >> 1;
  const bool up = (q.w & 1) != 0;
  T *Iray = I + (int64_t)(ray - ray0) * n * nl;
  const int64_t bi = (int64_t)site * nl, ei = (int64_t)site * cs;
  if (k1 < 0) {
    for (int l = l0; l < nl; l += C * V) {
      VT v;
      if (up) v = L::load(Ibot + ei + l);
      else if (Itop) v = L::load(Itop + ei + l);
      else v = VT(T(0));
      L::store(Iray + bi + l, v);
    }
    return;
  }
  const auto f = rf[rec];
  const T w1 = f.w1, w2 = T(1) - f.w1;
  const T h1 = T(0.5) * f.ds1, h2 = T(0.5) * f.ds2;
  const bool two = k2 >= 0;
  const int64_t b1 = (int64_t)k1 * nl;
  const int64_t b2 = (int64_t)(two ? k2 : k1) * nl;
  const int64_t e1 = (int64_t)k1 * cs, e2 = (int64_t)(two ? k2 : k1) * cs;
  for (int l = l0; l < nl; l += C * V) {
    const VT ci = L::load(chi + ei + l), si = L::load(S + ei + l);
    const VT c1 = L::load(chi + e1 + l), s1 = L::load(S + e1 + l), u1 = L::load(Iray + b1 + l);
    VT c2, s2, u2;
    if (two) {
      c2 = L::load(chi + e2 + l);
      s2 = L::load(S + e2 + l);
      u2 = L::load(Iray + b2 + l);
    }
    VT out;
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const T cik = L::get(ci, k), sik = L::get(si, k);
      T Iv = vrt::seg_line<T>((L::get(c1, k) + cik) * h1, L::get(u1, k), L::get(s1, k), sik);
      if (two) {
        const T Ib = vrt::seg_line<T>((L::get(c2, k) + cik) * h2, L::get(u2, k), L::get(s2, k), sik);
        Iv = vrt::seg_mix<T>(w1, w2, Iv, Ib);
      }
      L::set(out, k, Iv);
    }
    L::store(Iray + bi + l, out);
  }
}

// Single precision with lanes of at most 16 bytes: the body fits 64
// registers, so 8 wavefronts per SIMD stay resident (more gathers in flight
// per compute unit).
template <typename T, int C, int V>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void sweep_kernel(
    const int4 *__restrict__ ri, const typename vrt::RecOf<T>::type *__restrict__ rf, int64_t rec_begin,
    int64_t rec_count, int32_t nl, int64_t cs, int64_t n, const T *__restrict__ chi, const T *__restrict__ S,
    const T *__restrict__ Ibot, const T *__restrict__ Itop, T *I, int32_t xcd_chunks, int32_t ray0,
    const int64_t *__restrict__ xtab, int32_t xk) {
  sweep_body<T, C, V>(ri, rf, rec_begin, rec_count, nl, cs, n, chi, S, Ibot, Itop, I, xcd_chunks, ray0, xtab, xk);
}

// Double precision, or 32-byte lanes (twice the records per wavefront): more
// registers per wavefront, no occupancy bound
template <typename T, int C, int V>
__global__ __launch_bounds__(256) void sweep_kernel_wide(
    const int4 *__restrict__ ri, const typename vrt::RecOf<T>::type *__restrict__ rf, int64_t rec_begin,
    int64_t rec_count, int32_t nl, int64_t cs, int64_t n, const T *__restrict__ chi, const T *__restrict__ S,
    const T *__restrict__ Ibot, const T *__restrict__ Itop, T *I, int32_t xcd_chunks, int32_t ray0,
    const int64_t *__restrict__ xtab, int32_t xk) {
  sweep_body<T, C, V>(ri, rf, rec_begin, rec_count, nl, cs, n, chi, S, Ibot, Itop, I, xcd_chunks, ray0, xtab, xk);
}

// Pipelined form of the same update for interior records (level steps >= 1:
// step 0 holds exactly the boundary sites), for rows of at most C*V
// wavelengths (one lane-vector per lane). A launch of classic wavefronts is
// bound by latency, not by bandwidth or arithmetic: each wavefront runs one
// dependent chain (its records, then the rows they name, then the update) and
// ends, and with eight wavefronts per SIMD too few loads are in flight. Here a
// wavefront sweeps Q consecutive groups of 64/C records, fully unrolled: the
// records of group j + 2 and the rows of group j + 1 are issued before group j
// is computed, so the in-order completion of vector loads lets each wait cover
// only what it needs. The code has no branches between the loads and their
// uses (both lines are always formed, then selected; records past the range and
// lanes past the row clamp their loads to valid addresses and store the same
// bits as the lane that owns the element), because a join of divergent paths
// makes the compiler wait for every load in flight. The arithmetic per record is the classic kernel's: same bits.
template <typename T, int C, int V, int Q>
__global__ __launch_bounds__(256) void sweep_pipe_kernel(
    const int4 *__restrict__ ri, const typename vrt::RecOf<T>::type *__restrict__ rf, int64_t rec_begin,
    int64_t rec_count, int32_t nl, int64_t cs, int64_t n, const T *__restrict__ chi, const T *__restrict__ S, T *I,
    int32_t xcd_chunks) {
  using L = Lane<T, V>;
  using VT = typename L::type;
  using RF = typename vrt::RecOf<T>::type;
  constexpr int SPW = 64 / C;
  const int lane = threadIdx.x & 63;
  const int lv = (lane % C) * V;
  const int l = lv < nl ? lv : nl - V;  // a lane past the row re-reads the last vector
  const int64_t wave = chunked_block(xcd_chunks) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t first = wave * (int64_t)(SPW * Q) + lane / C;
  int4 q[Q];
  RF f[Q];
  VT ci[Q], si[Q], c1[Q], s1[Q], u1[Q], c2[Q], s2[Q], u2[Q];
  auto load_rec = [&](int j) {
    const int64_t r = first + (int64_t)j * SPW;
    const int64_t rc = rec_begin + (r < rec_count ? r : rec_count - 1);
    q[j] = ri[rc];
    f[j] = rf[rc];
  };
  auto load_rows = [&](int j) {
    // a missing second line reads the first again; indices are clamped so that
    // no load leaves the arrays even for a record this kernel does not expect
    const int32_t k1 = q[j].y > 0 ? q[j].y : 0;
    const int32_t k2 = q[j].z >= 0 ? q[j].z : k1;
    T *Iray = I + (int64_t)(q[j].w >> 1) * n * nl;
    const int64_t b1 = (int64_t)k1 * nl + l, b2 = (int64_t)k2 * nl + l;
    const int64_t ei = (int64_t)q[j].x * cs + l, e1 = (int64_t)k1 * cs + l, e2 = (int64_t)k2 * cs + l;
    ci[j] = L::load(chi + ei);
    si[j] = L::load(S + ei);
    c1[j] = L::load(chi + e1);
    s1[j] = L::load(S + e1);
    u1[j] = L::load(Iray + b1);
    c2[j] = L::load(chi + e2);
    s2[j] = L::load(S + e2);
    u2[j] = L::load(Iray + b2);
  };
  auto finish = [&](int j) {
    const T w1 = f[j].w1, w2 = T(1) - f[j].w1;
    const T h1 = T(0.5) * f[j].ds1, h2 = T(0.5) * f[j].ds2;
    const bool two = q[j].z >= 0;
    VT out;
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const T cik = L::get(ci[j], k), sik = L::get(si[j], k);
      const T Ia = vrt::seg_line<T>((L::get(c1[j], k) + cik) * h1, L::get(u1[j], k), L::get(s1[j], k), sik);
      const T Ib = vrt::seg_line<T>((L::get(c2[j], k) + cik) * h2, L::get(u2[j], k), L::get(s2[j], k), sik);
      const T Im = vrt::seg_mix<T>(w1, w2, Ia, Ib);
      L::set(out, k, two ? Im : Ia);
    }
    // unconditional: a lane past the range holds the last record and a lane
    // past the row the row's last vector, so it writes the very bits the
    // owning lane writes (a guarded store would let the compiler sink this
    // group's loads into the guard, after the previous group's compute)
    L::store(I + (int64_t)(q[j].w >> 1) * n * nl + (int64_t)q[j].x * nl + l, out);
  };
  // scheduling barriers keep each stage's loads ahead of the previous group's
  // arithmetic (left alone, the scheduler moves loads next to their uses to
  // save registers, which serialises the groups again)
  load_rec(0);
  if (Q > 1) load_rec(1);
  load_rows(0);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    if (j + 2 < Q) load_rec(j + 2);
    if (j + 1 < Q) load_rows(j + 1);
    __builtin_amdgcn_sched_barrier(0);
    finish(j);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// J = sum_r w_r I_r with double accumulation (ray order fixed); V elements per thread.
// ABS reads sign-encoded rows (the persistent sweep's epoch sign) as |I|; if
// the sweep's device error word is set, those rows are not this epoch's (the
// sweep stopped early or did not run), and J is written as NaN instead.
template <typename T, int V, bool ABS>
__global__ __launch_bounds__(256) void jreduce_kernel(const T *__restrict__ I, int32_t R, int64_t nn,
                                                      const double *__restrict__ w, T *__restrict__ J,
                                                      const int32_t *__restrict__ err) {
  using L = Lane<T, V>;
  using VT = typename L::type;
  const int64_t nv = nn / V;
  if (ABS && err && *err != 0) {
    VT nan;
#pragma unroll
    for (int k = 0; k < V; ++k) L::set(nan, k, (T)__builtin_nan(""));
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nv; t += (int64_t)gridDim.x * blockDim.x)
      L::store(J + t * V, nan);
    return;
  }
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nv; t += (int64_t)gridDim.x * blockDim.x) {
    double acc[V];
#pragma unroll
    for (int k = 0; k < V; ++k) acc[k] = 0.0;
    // rays in order, eight loads in flight before their sums (each intensity
    // is read once: non-temporal streaming loads)
    auto add = [&](const VT &x, double wr) {
#pragma unroll
      for (int k = 0; k < V; ++k) acc[k] += wr * (ABS ? __builtin_fabs((double)L::get(x, k)) : (double)L::get(x, k));
    };
    int32_t r = 0;
    for (; r + 8 <= R; r += 8) {
      VT x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        x[u] = __builtin_nontemporal_load(reinterpret_cast<const VT *>(I + (int64_t)(r + u) * nn + t * V));
#pragma unroll
      for (int u = 0; u < 8; ++u) add(x[u], w[r + u]);
    }
    for (; r < R; ++r) add(__builtin_nontemporal_load(reinterpret_cast<const VT *>(I + (int64_t)r * nn + t * V)), w[r]);
    VT out;
#pragma unroll
    for (int k = 0; k < V; ++k) L::set(out, k, (T)acc[k]);
    L::store(J + t * V, out);
  }
}

// I rows have ld >= nl entries; out rows have nl.
// C lanes per emergent row (a power of two), 64/C rows per wavefront, V
// consecutive wavelengths (16 bytes) per lane when the rows allow it. ABS:
// sign-encoded rows, NaN when the sweep's device error word is set (as in J).
template <typename T, int C, int V, bool ABS>
__global__ __launch_bounds__(256) void emergent_kernel(int64_t total, int32_t nl, int32_t ld, int64_t n,
                                                       const int32_t *__restrict__ em_ray,
                                                       const int32_t *__restrict__ em_site, const T *__restrict__ I,
                                                       T *__restrict__ out, const int32_t *__restrict__ err) {
  using L = Lane<T, V>;
  constexpr int SPW = 64 / C;
  const int lane = threadIdx.x & 63;
  const int64_t e = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * SPW + lane / C;
  if (e >= total) return;
  const bool stale = ABS && err && *err != 0;
  const T *src = I + ((int64_t)em_ray[e] * n + em_site[e]) * ld;
  T *dst = out + e * nl;
  for (int32_t l = (lane % C) * V; l < nl; l += C * V) {
    auto x = L::load(src + l);
    if constexpr (ABS) {
#pragma unroll
      for (int k = 0; k < V; ++k)
        L::set(x, k, stale ? (T)__builtin_nan("") : (T)__builtin_fabs((double)L::get(x, k)));
    }
    L::store(dst + l, x);
  }
}

template <typename T, int C, int V>
void launch_ec(hipStream_t s, int64_t total, int32_t nl, int32_t ld, int64_t n, const int32_t *em_ray,
               const int32_t *em_site, const T *I, T *out, bool ab, const int32_t *err) {
  constexpr int SPW = 64 / C;
  const int64_t blocks = (total + 4 * SPW - 1) / (4 * SPW);
  auto kern = ab ? emergent_kernel<T, C, V, true> : emergent_kernel<T, C, V, false>;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, s, total, nl, ld, n, em_ray, em_site, I, out, err);
}

template <typename T, int V>
void launch_ev(hipStream_t s, int64_t total, int32_t nl, int32_t ld, int64_t n, const int32_t *em_ray,
               const int32_t *em_site, const T *I, T *out, bool ab, const int32_t *err) {
  switch (vrt::lanes_per_record(nl / V)) {
    case 64: launch_ec<T, 64, V>(s, total, nl, ld, n, em_ray, em_site, I, out, ab, err); break;
    case 32: launch_ec<T, 32, V>(s, total, nl, ld, n, em_ray, em_site, I, out, ab, err); break;
    case 16: launch_ec<T, 16, V>(s, total, nl, ld, n, em_ray, em_site, I, out, ab, err); break;
    case 8: launch_ec<T, 8, V>(s, total, nl, ld, n, em_ray, em_site, I, out, ab, err); break;
    case 4: launch_ec<T, 4, V>(s, total, nl, ld, n, em_ray, em_site, I, out, ab, err); break;
    case 2: launch_ec<T, 2, V>(s, total, nl, ld, n, em_ray, em_site, I, out, ab, err); break;
    default: launch_ec<T, 1, V>(s, total, nl, ld, n, em_ray, em_site, I, out, ab, err); break;
  }
}

// With a ray-affinity table, c is the largest record count of one die and the
// grid holds that many records for every die.
template <typename T, int C, int V, int Q>
void launch_pipe(hipStream_t s, const int4 *ri, const typename vrt::RecOf<T>::type *rf, int64_t b, int64_t c,
                 int32_t nl, int64_t cs, int64_t n, const T *chi, const T *S, T *I, int32_t xc) {
  constexpr int SPW = 64 / C;
  const int64_t waves = (c + SPW * Q - 1) / (SPW * Q);
  const int64_t blocks = (waves + 3) / 4;
  hipLaunchKernelGGL((sweep_pipe_kernel<T, C, V, Q>), dim3((unsigned)blocks), dim3(256), 0, s, ri, rf, b, c, nl, cs,
                     n, chi, S, I, xc);
}

template <typename T, int C, int V>
void launch_c(hipStream_t s, const int4 *ri, const typename vrt::RecOf<T>::type *rf, int64_t b, int64_t c, int32_t nl,
              int64_t cs, int64_t n, const T *chi, const T *S, const T *Ibot, const T *Itop, T *I, int32_t xc,
              int32_t ray0, const int64_t *xtab, int32_t xk, int32_t pipe) {
  constexpr int SPW = 64 / C;
  if constexpr (V * sizeof(T) == 16) {
    // the pipelined kernel (pipe > 0 is passed only for interior level steps):
    // per-ray rows from I (ray0 = 0), no affinity table, one lane-vector per lane
    if (pipe > 0 && !xtab && ray0 == 0 && nl <= C * V) {
      if (pipe >= 8) launch_pipe<T, C, V, 8>(s, ri, rf, b, c, nl, cs, n, chi, S, I, xc);
      else if (pipe >= 4) launch_pipe<T, C, V, 4>(s, ri, rf, b, c, nl, cs, n, chi, S, I, xc);
      else launch_pipe<T, C, V, 2>(s, ri, rf, b, c, nl, cs, n, chi, S, I, xc);
      return;
    }
  }
  const int64_t waves = (c + SPW - 1) / SPW;
  const int64_t blocks = xtab ? (int64_t)vrt::kDies * ((waves + 3) / 4) : (waves + 3) / 4;
  if constexpr (sizeof(T) != 4 || V * sizeof(T) > 16)
    hipLaunchKernelGGL((sweep_kernel_wide<T, C, V>), dim3((unsigned)blocks), dim3(256), 0, s, ri, rf, b, c, nl, cs, n,
                       chi, S, Ibot, Itop, I, xc, ray0, xtab, xk);
  else
    hipLaunchKernelGGL((sweep_kernel<T, C, V>), dim3((unsigned)blocks), dim3(256), 0, s, ri, rf, b, c, nl, cs, n, chi,
                       S, Ibot, Itop, I, xc, ray0, xtab, xk);
}

// lanes per record for m lane-vectors per row: the smallest power of two >= m, at most 64
template <typename T, int V>
void launch_v(hipStream_t s, const int4 *ri, const typename vrt::RecOf<T>::type *rf, int64_t b, int64_t c, int32_t nl,
              int64_t cs, int64_t n, const T *chi, const T *S, const T *Ibot, const T *Itop, T *I, int32_t xc,
              int32_t ray0, const int64_t *xtab, int32_t xk, int32_t pp) {
  const int32_t m = nl / V;
  if (m >= 33) launch_c<T, 64, V>(s, ri, rf, b, c, nl, cs, n, chi, S, Ibot, Itop, I, xc, ray0, xtab, xk, pp);
  else if (m >= 17) launch_c<T, 32, V>(s, ri, rf, b, c, nl, cs, n, chi, S, Ibot, Itop, I, xc, ray0, xtab, xk, pp);
  else if (m >= 9) launch_c<T, 16, V>(s, ri, rf, b, c, nl, cs, n, chi, S, Ibot, Itop, I, xc, ray0, xtab, xk, pp);
  else if (m >= 5) launch_c<T, 8, V>(s, ri, rf, b, c, nl, cs, n, chi, S, Ibot, Itop, I, xc, ray0, xtab, xk, pp);
  else if (m >= 3) launch_c<T, 4, V>(s, ri, rf, b, c, nl, cs, n, chi, S, Ibot, Itop, I, xc, ray0, xtab, xk, pp);
  else if (m == 2) launch_c<T, 2, V>(s, ri, rf, b, c, nl, cs, n, chi, S, Ibot, Itop, I, xc, ray0, xtab, xk, pp);
  else launch_c<T, 1, V>(s, ri, rf, b, c, nl, cs, n, chi, S, Ibot, Itop, I, xc, ray0, xtab, xk, pp);
}

// Forward sweep with checkpointed intensities, for the reverse sweep: the rows
// of one ray group do not live at their site's index but in two compact
// buffers, a chunk buffer Ich holding the rows of the level chunk being swept
// and a frontier buffer Ifr holding, for every later chunk, the rows it reads
// from earlier chunks. ck[rec] = {chunk slot of the record, frontier slot or
// -1, location of the upwind row of line 1, of line 2}; a location >= 0 is a
// chunk slot, -(f + 1) frontier slot f. The update is the arithmetic of
// sweep_body, so the rows are bit-identical to an unchecked sweep's.
template <typename T, int C, int V>
__global__ __launch_bounds__(256) void ck_sweep_kernel(const int4 *__restrict__ ri,
                                                       const typename vrt::RecOf<T>::type *__restrict__ rf,
                                                       const int4 *__restrict__ ck, int64_t rec_begin,
                                                       int64_t rec_count, int32_t nl, const T *__restrict__ chi,
                                                       const T *__restrict__ S, const T *__restrict__ Ibot,
                                                       const T *__restrict__ Itop, T *Ich, T *Ifr) {
  using L = Lane<T, V>;
  using VT = typename L::type;
  constexpr int SPW = 64 / C;
  const int lane = threadIdx.x & 63;
  const int l0 = (lane % C) * V;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t r = wave * SPW + lane / C;
  if (r >= rec_count) return;
  const int64_t rec = rec_begin + r;
  const int4 q = ri[rec];
  const int4 t = ck[rec];
  const int32_t site = q.x, k1 = q.y, k2 = q.z;
  const bool up = (q.w & 1) != 0;
  T *own = Ich + (int64_t)t.x * nl;
  T *fr = t.y >= 0 ? Ifr + (int64_t)t.y * nl : nullptr;
  const int64_t bi = (int64_t)site * nl;
  if (k1 < 0) {
    for (int l = l0; l < nl; l += C * V) {
      VT v;
      if (up) v = L::load(Ibot + bi + l);
      else if (Itop) v = L::load(Itop + bi + l);
      else v = VT(T(0));
      L::store(own + l, v);
      if (fr) L::store(fr + l, v);
    }
    return;
  }
  const auto f = rf[rec];
  const T w1 = f.w1, w2 = T(1) - f.w1;
  const T h1 = T(0.5) * f.ds1, h2 = T(0.5) * f.ds2;
  const bool two = k2 >= 0;
  const int64_t b1 = (int64_t)k1 * nl;
  const int64_t b2 = (int64_t)(two ? k2 : k1) * nl;
  const T *p1 = t.z >= 0 ? Ich + (int64_t)t.z * nl : Ifr + (int64_t)(-t.z - 1) * nl;
  const T *p2 = t.w >= 0 ? Ich + (int64_t)t.w * nl : Ifr + (int64_t)(-t.w - 1) * nl;
  for (int l = l0; l < nl; l += C * V) {
    const VT ci = L::load(chi + bi + l), si = L::load(S + bi + l);
    const VT c1 = L::load(chi + b1 + l), s1 = L::load(S + b1 + l), u1 = L::load(p1 + l);
    VT c2, s2, u2;
    if (two) {
      c2 = L::load(chi + b2 + l);
      s2 = L::load(S + b2 + l);
      u2 = L::load(p2 + l);
    }
    VT out;
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const T cik = L::get(ci, k), sik = L::get(si, k);
      T Iv = vrt::seg_line<T>((L::get(c1, k) + cik) * h1, L::get(u1, k), L::get(s1, k), sik);
      if (two) {
        const T Ib = vrt::seg_line<T>((L::get(c2, k) + cik) * h2, L::get(u2, k), L::get(s2, k), sik);
        Iv = vrt::seg_mix<T>(w1, w2, Iv, Ib);
      }
      L::set(out, k, Iv);
    }
    L::store(own + l, out);
    if (fr) L::store(fr + l, out);
  }
}

template <typename T, int V>
void launch_ckv(hipStream_t s, const int4 *ri, const typename vrt::RecOf<T>::type *rf, const int4 *ck, int64_t b,
                int64_t c, int32_t nl, const T *chi, const T *S, const T *Ibot, const T *Itop, T *Ich, T *Ifr) {
#define VRT_CKC(CC)                                                                                                  \
  hipLaunchKernelGGL((ck_sweep_kernel<T, CC, V>), dim3((unsigned)(((c + 64 / CC - 1) / (64 / CC) + 3) / 4)),        \
                     dim3(256), 0, s, ri, rf, ck, b, c, nl, chi, S, Ibot, Itop, Ich, Ifr)
  switch (vrt::lanes_per_record(nl / V)) {
    case 64: VRT_CKC(64); break;
    case 32: VRT_CKC(32); break;
    case 16: VRT_CKC(16); break;
    case 8: VRT_CKC(8); break;
    case 4: VRT_CKC(4); break;
    case 2: VRT_CKC(2); break;
    default: VRT_CKC(1); break;
  }
#undef VRT_CKC
}

// 16-byte lane vectors when the row length allows (and rows then stay 16-byte aligned)
template <typename T> constexpr int kVec = 16 / sizeof(T);

inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
inline bool aligned32p(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 31u) == 0; }

}  // namespace

namespace vrt {

template <typename T>
void launch_sweep(hipStream_t s, const int4 *ri, const typename RecOf<T>::type *rf, int64_t rec_begin,
                  int64_t rec_count, int32_t nl, int64_t cs, int64_t n, const T *chi, const T *S, const T *Ibot,
                  const T *Itop, T *I, int32_t xcd_chunks, int32_t ray0, const int64_t *xtab, int32_t xk,
                  int32_t lane_bytes, int32_t pipe) {
  if (rec_count <= 0) return;
  // a vector lane needs every row it reads to start on its own boundary: the
  // row lengths and the chi / S row stride are multiples of the vector width
  const bool aligned = aligned16(chi) && aligned16(S) && aligned16(Ibot) && aligned16(Itop) && aligned16(I);
  const bool aligned32 = aligned32p(chi) && aligned32p(S) && aligned32p(Ibot) && aligned32p(Itop) && aligned32p(I);
  if (lane_bytes == 32 && aligned32 && nl % (2 * kVec<T>) == 0 && cs % (2 * kVec<T>) == 0)
    launch_v<T, 2 * kVec<T>>(s, ri, rf, rec_begin, rec_count, nl, cs, n, chi, S, Ibot, Itop, I, xcd_chunks, ray0,
                             xtab, xk, 0);
  else if (aligned && nl % kVec<T> == 0 && cs % kVec<T> == 0)
    launch_v<T, kVec<T>>(s, ri, rf, rec_begin, rec_count, nl, cs, n, chi, S, Ibot, Itop, I, xcd_chunks, ray0, xtab,
                         xk, pipe);
  else
    launch_v<T, 1>(s, ri, rf, rec_begin, rec_count, nl, cs, n, chi, S, Ibot, Itop, I, xcd_chunks, ray0, xtab, xk, 0);
  VRT_HIP(hipGetLastError());
}

template <typename T>
void launch_sweep_ck(hipStream_t s, const int4 *ri, const typename RecOf<T>::type *rf, const int4 *ck,
                     int64_t rec_begin, int64_t rec_count, int32_t nl, const T *chi, const T *S, const T *Ibot,
                     const T *Itop, T *Ich, T *Ifr) {
  if (rec_count <= 0) return;
  const bool aligned =
      aligned16(chi) && aligned16(S) && aligned16(Ibot) && aligned16(Itop) && aligned16(Ich) && aligned16(Ifr);
  if (aligned && nl % kVec<T> == 0)
    launch_ckv<T, kVec<T>>(s, ri, rf, ck, rec_begin, rec_count, nl, chi, S, Ibot, Itop, Ich, Ifr);
  else
    launch_ckv<T, 1>(s, ri, rf, ck, rec_begin, rec_count, nl, chi, S, Ibot, Itop, Ich, Ifr);
  VRT_HIP(hipGetLastError());
}

template <typename T>
void launch_jreduce(hipStream_t s, const T *I, int32_t R, int64_t nn, const double *w, T *J, bool abs_rows,
                    const int32_t *err) {
  if (nn == 0) return;
  const bool vec = nn % kVec<T> == 0 && aligned16(I) && aligned16(J);
  const int64_t items = vec ? nn / kVec<T> : nn;
  int64_t blocks = (items + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  auto kern = vec ? (abs_rows ? jreduce_kernel<T, kVec<T>, true> : jreduce_kernel<T, kVec<T>, false>)
                  : (abs_rows ? jreduce_kernel<T, 1, true> : jreduce_kernel<T, 1, false>);
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, s, I, R, nn, w, J, err);
  VRT_HIP(hipGetLastError());
}

template <typename T>
void launch_emergent(hipStream_t s, int64_t total, int32_t nl, int32_t ld, int64_t n, const int32_t *em_ray,
                     const int32_t *em_site, const T *I, T *out, bool abs_rows, const int32_t *err) {
  if (total == 0 || nl == 0) return;
  if (nl % kVec<T> == 0 && ld % kVec<T> == 0 && aligned16(I) && aligned16(out))
    launch_ev<T, kVec<T>>(s, total, nl, ld, n, em_ray, em_site, I, out, abs_rows, err);
  else
    launch_ev<T, 1>(s, total, nl, ld, n, em_ray, em_site, I, out, abs_rows, err);
  VRT_HIP(hipGetLastError());
}

template void launch_sweep<float>(hipStream_t, const int4 *, const RecF32 *, int64_t, int64_t, int32_t, int64_t,
                                  int64_t, const float *, const float *, const float *, const float *, float *,
                                  int32_t, int32_t, const int64_t *, int32_t, int32_t, int32_t);
template void launch_sweep<double>(hipStream_t, const int4 *, const RecF64 *, int64_t, int64_t, int32_t, int64_t,
                                   int64_t, const double *, const double *, const double *, const double *, double *,
                                   int32_t, int32_t, const int64_t *, int32_t, int32_t, int32_t);
template void launch_sweep_ck<float>(hipStream_t, const int4 *, const RecF32 *, const int4 *, int64_t, int64_t,
                                     int32_t, const float *, const float *, const float *, const float *, float *,
                                     float *);
template void launch_sweep_ck<double>(hipStream_t, const int4 *, const RecF64 *, const int4 *, int64_t, int64_t,
                                      int32_t, const double *, const double *, const double *, const double *,
                                      double *, double *);
template void launch_jreduce<float>(hipStream_t, const float *, int32_t, int64_t, const double *, float *, bool,
                                    const int32_t *);
template void launch_jreduce<double>(hipStream_t, const double *, int32_t, int64_t, const double *, double *,
                                     bool, const int32_t *);
template void launch_emergent<float>(hipStream_t, int64_t, int32_t, int32_t, int64_t, const int32_t *,
                                     const int32_t *, const float *, float *, bool, const int32_t *);
template void launch_emergent<double>(hipStream_t, int64_t, int32_t, int32_t, int64_t, const int32_t *,
                                      const int32_t *, const double *, double *, bool, const int32_t *);

}  // namespace vrt
