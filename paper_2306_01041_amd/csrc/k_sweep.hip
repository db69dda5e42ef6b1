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

template <typename T, int C>
__global__ __launch_bounds__(256) void sweep_kernel(const int4 *__restrict__ ri,
                                                    const typename vrt::RecOf<T>::type *__restrict__ rf,
                                                    int64_t rec_begin, int64_t rec_count, int32_t nl, int64_t n,
                                                    const T *__restrict__ chi, const T *__restrict__ S,
                                                    const T *__restrict__ Ibot, const T *__restrict__ Itop, T *I) {
  constexpr int SPW = 64 / C;
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t rec = wave * SPW + lane / C;
  const int l0 = lane % C;
  if (rec >= rec_count) return;
  const int4 q = ri[rec_begin + rec];
  const int32_t site = q.x, k1 = q.y, k2 = q.z;
  const int32_t ray = q.w >> 1;
  const bool up = (q.w & 1) != 0;
  T *Iray = I + (int64_t)ray * n * nl;
  const int64_t bi = (int64_t)site * nl;
  if (k1 < 0) {
    for (int l = l0; l < nl; l += C) {
      T v = T(0);
      if (up) v = Ibot[bi + l];
      else if (Itop) v = Itop[bi + l];
      Iray[bi + l] = v;
    }
    return;
  }
  const auto f = rf[rec_begin + rec];
  const T w1 = f.w1, w2 = T(1) - f.w1;
  const T h1 = T(0.5) * f.ds1, h2 = T(0.5) * f.ds2;
  const int64_t b1 = (int64_t)k1 * nl;
  const int64_t b2 = (int64_t)(k2 >= 0 ? k2 : k1) * nl;
  for (int l = l0; l < nl; l += C) {
    const T ci = chi[bi + l], si = S[bi + l];
    T E, pu, p0;
    vrt::Seg<T>::weights((chi[b1 + l] + ci) * h1, E, pu, p0);
    const T Ia = E * Iray[b1 + l] + pu * S[b1 + l] + p0 * si;
    T Iv = Ia;
    if (k2 >= 0) {
      vrt::Seg<T>::weights((chi[b2 + l] + ci) * h2, E, pu, p0);
      const T Ib = E * Iray[b2 + l] + pu * S[b2 + l] + p0 * si;
      Iv = w1 * Ia + w2 * Ib;
    }
    Iray[bi + l] = Iv;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void jreduce_kernel(const T *__restrict__ I, int32_t R, int64_t nn,
                                                      const double *__restrict__ w, T *__restrict__ J) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nn; t += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int32_t r = 0; r < R; ++r) acc += w[r] * (double)I[(int64_t)r * nn + t];
    J[t] = (T)acc;
  }
}

template <typename T>
__global__ void emergent_kernel(int64_t total, int32_t nl, int64_t n, const int32_t *__restrict__ em_ray,
                                const int32_t *__restrict__ em_site, const T *__restrict__ I, T *__restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total * nl) return;
  const int64_t e = t / nl;
  const int32_t l = (int32_t)(t - e * nl);
  out[t] = I[((int64_t)em_ray[e] * n + em_site[e]) * nl + l];
}

template <typename T, int C>
void launch_c(hipStream_t s, const int4 *ri, const typename vrt::RecOf<T>::type *rf, int64_t b, int64_t c, int32_t nl,
              int64_t n, const T *chi, const T *S, const T *Ibot, const T *Itop, T *I) {
  constexpr int SPW = 64 / C;
  const int64_t waves = (c + SPW - 1) / SPW;
  const int64_t blocks = (waves + 3) / 4;
  hipLaunchKernelGGL((sweep_kernel<T, C>), dim3((unsigned)blocks), dim3(256), 0, s, ri, rf, b, c, nl, n, chi, S,
                     Ibot, Itop, I);
}

}  // namespace

namespace vrt {

template <typename T>
void launch_sweep(hipStream_t s, const int4 *ri, const typename RecOf<T>::type *rf, int64_t rec_begin,
                  int64_t rec_count, int32_t nl, int64_t n, const T *chi, const T *S, const T *Ibot, const T *Itop,
                  T *I) {
  if (rec_count <= 0) return;
  if (nl >= 33) launch_c<T, 64>(s, ri, rf, rec_begin, rec_count, nl, n, chi, S, Ibot, Itop, I);
  else if (nl >= 17) launch_c<T, 32>(s, ri, rf, rec_begin, rec_count, nl, n, chi, S, Ibot, Itop, I);
  else if (nl >= 9) launch_c<T, 16>(s, ri, rf, rec_begin, rec_count, nl, n, chi, S, Ibot, Itop, I);
  else if (nl >= 5) launch_c<T, 8>(s, ri, rf, rec_begin, rec_count, nl, n, chi, S, Ibot, Itop, I);
  else if (nl >= 3) launch_c<T, 4>(s, ri, rf, rec_begin, rec_count, nl, n, chi, S, Ibot, Itop, I);
  else if (nl == 2) launch_c<T, 2>(s, ri, rf, rec_begin, rec_count, nl, n, chi, S, Ibot, Itop, I);
  else launch_c<T, 1>(s, ri, rf, rec_begin, rec_count, nl, n, chi, S, Ibot, Itop, I);
  VRT_HIP(hipGetLastError());
}

template <typename T>
void launch_jreduce(hipStream_t s, const T *I, int32_t R, int64_t nn, const double *w, T *J) {
  if (nn == 0) return;
  int64_t blocks = (nn + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(jreduce_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, I, R, nn, w, J);
  VRT_HIP(hipGetLastError());
}

template <typename T>
void launch_emergent(hipStream_t s, int64_t total, int32_t nl, int64_t n, const int32_t *em_ray,
                     const int32_t *em_site, const T *I, T *out) {
  const int64_t work = total * nl;
  if (work == 0) return;
  hipLaunchKernelGGL(emergent_kernel<T>, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, total, nl, n, em_ray,
                     em_site, I, out);
  VRT_HIP(hipGetLastError());
}

template void launch_sweep<float>(hipStream_t, const int4 *, const RecF32 *, int64_t, int64_t, int32_t, int64_t,
                                  const float *, const float *, const float *, const float *, float *);
template void launch_sweep<double>(hipStream_t, const int4 *, const RecF64 *, int64_t, int64_t, int32_t, int64_t,
                                   const double *, const double *, const double *, const double *, double *);
template void launch_jreduce<float>(hipStream_t, const float *, int32_t, int64_t, const double *, float *);
template void launch_jreduce<double>(hipStream_t, const double *, int32_t, int64_t, const double *, double *);
template void launch_emergent<float>(hipStream_t, int64_t, int32_t, int64_t, const int32_t *, const int32_t *,
                                     const float *, float *);
template void launch_emergent<double>(hipStream_t, int64_t, int32_t, int64_t, const int32_t *, const int32_t *,
                                      const double *, double *);

}  // namespace vrt
