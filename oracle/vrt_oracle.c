/*
 * vrt_oracle.c -- plain, slow, FP64 CPU reference of the formal solution on
 * irregular (Voronoi) and regular grids.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do. It shares no code, header or constant with the HIP
 * library. Every loop is written in the order the method defines it; there is
 * no blocking, fusion or level scheduling (sites are swept in plain height
 * order, which is a valid upwind order because every dependency lies strictly
 * upwind in z).
 *
 * Method (Udnaes & Pereira 2023, arXiv:2306.01041):
 *   - RTE along a ray, dI/dtau = S - I                        (Sect. 2.1, Eq. 1)
 *   - formal solution I = I0 e^-tau + int S e^-(tau-t) dt       (Sect. 2.1, Eq. 2)
 *     discretised with S linear along each segment              (Sect. 2.5)
 *   - intensity at a site from the two Delaunay lines closest
 *     to the ray, I_i = w1 I_i1 + w2 I_i2                       (Sect. 2.5, Eq. 5)
 *   - w_j = v_j^r / (v_1^r + v_2^r), v = cosine between ray and
 *     Delaunay line, r = 7                                      (Sect. 2.5, Eq. 6)
 *   - rays start at the bottom (upward) or top (downward)       (Sect. 2.5)
 *   - J = angle quadrature of I                                 (Sect. 2.1, Eq. 4)
 *   - regular-grid short characteristics with linear
 *     interpolation                                             (Sect. 2.6)
 *
 * Readings where the paper is silent (the same list is kept in the design
 * notes of the repository):
 *   R1 candidates for site i on a ray n with sigma = sign(n_z): neighbours k
 *      strictly upwind in height (sigma*(z_i - z_k) > 0) with n.d > 0, where
 *      d = r_i - (r_k + shift*L) is the Delaunay line pointing into i;
 *   R2 ranking key q = (n.d)|n.d| / |d|^2 (same order as v = n.d/|d|),
 *      computed with +,-,*,/ in a fixed order and no fused multiply-add; ties
 *      go to the smaller neighbour index, then to the earlier CSR entry;
 *   R3 one candidate -> weight 1; none -> the z-upwind neighbour with the
 *      largest key, weight 1 (a "fallback");
 *   R4 a site whose cell touches the upwind z-wall is a boundary site: it
 *      takes I_bottom (upward rays) or I_top (downward rays, default 0);
 *   R5 path length along line j is |d_j|; optical depth of the segment is the
 *      trapezoid x = (chi_k + chi_i)/2 * |d_j|;
 *   R6 regular grid: the upwind point lies in the adjacent horizontal plane,
 *      periodic bilinear interpolation of I, S and chi there, path length
 *      dz/|mu|.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * Segment weights for S linear along a segment of optical depth x
 * (Sect. 2.5, linear interpolation of S inside Eq. 2):
 *   I = e^-x I_u + Psi_u S_u + Psi_0 S_0,
 *   e0 = 1 - e^-x, e1 = x - e0, Psi_0 = e1/x, Psi_u = e0 - e1/x.
 * For x < 1/2 the ratios are summed from their power series,
 *   Psi_0 = sum_{n>=1} (-1)^(n+1) x^n/(n+1)!,
 *   Psi_u = sum_{n>=1} (-1)^(n+1) n x^n/(n+1)!,
 * which avoids the cancellation in e1 and the 0/0 at x = 0. For x >= 1/2 the
 * same closed form is evaluated as Psi_0 = 1 - e0/x and Psi_u = e0/x - e^-x
 * (identical algebraically), which does not cancel when x is large.
 * ------------------------------------------------------------------------- */
void orc_psi(double x, double *E, double *psi_u, double *psi_0) {
    if (x < 0.5) {
        double term = 0.5 * x; /* n = 1: x/2! */
        double s0 = 0.0, su = 0.0;
        for (int n = 1; n <= 40; ++n) {
            s0 += term;
            su += (double)n * term;
            term *= -x / (double)(n + 2);
        }
        *E = exp(-x);
        *psi_0 = s0;
        *psi_u = su;
    } else {
        const double e = exp(-x);
        const double e0 = -expm1(-x);
        *E = e;
        *psi_0 = 1.0 - e0 / x;
        *psi_u = e0 / x - e;
    }
}

/* Derivatives of Psi_0 and Psi_u with respect to x (used by the reverse sweep).
 *   dPsi_0/dx = e0/x - e1/x^2 = sum_{n>=1} (-1)^(n+1) n x^(n-1)/(n+1)!
 *   dPsi_u/dx = e^-x - dPsi_0/dx
 */
void orc_dpsi(double x, double *dpsi_u, double *dpsi_0) {
    double d0;
    if (x < 0.5) {
        double s = 0.0;
        double p = 0.5; /* x^(n-1)/(n+1)! for n = 1 */
        for (int n = 1; n <= 40; ++n) {
            const double term = (double)n * p;
            s += (n % 2 == 1) ? term : -term;
            p *= x / (double)(n + 2);
        }
        d0 = s;
    } else {
        /* e0/x - e1/x^2 with e1 = x - e0 is e0/x^2 - (1 - e0)/x = (e0/x - e^-x)/x */
        const double e0 = -expm1(-x);
        d0 = (e0 / x - exp(-x)) / x;
    }
    *dpsi_0 = d0;
    *dpsi_u = exp(-x) - d0;
}

/* ---------------------------------------------------------------------------
 * Upwind selection (Sect. 2.5, Eq. 5-6; readings R1-R5).
 * Per ray r and site i: k1, k2 (caller indices, -1 = none), w1 (weight of
 * k1; w2 = 1 - w1), ds1, ds2 (line lengths). Boundary sites get k1 = k2 = -1.
 * Returns 0, or -2 if a non-boundary site has no z-upwind neighbour, or -1
 * for a horizontal ray.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t k;
    int64_t e;
    double q, dot, len2;
} orc_cand;

/* a ranks before b: larger key, then smaller neighbour index, then earlier entry */
static int orc_before(const orc_cand *a, const orc_cand *b) {
    if (a->q != b->q) return a->q > b->q;
    if (a->k != b->k) return a->k < b->k;
    return a->e < b->e;
}

int orc_select(int64_t n, const double *xyz, const int64_t *nbr_ptr, const int32_t *nbr_idx,
               const int8_t *nbr_shift, const uint8_t *wall, double Lx, double Ly, int32_t n_rays,
               const double *dirs, double r_exp, int32_t *k1, int32_t *k2, double *w1, double *ds1,
               double *ds2, int64_t *n_fallback) {
    int status = 0;
    for (int32_t r = 0; r < n_rays; ++r) {
        const double nx = dirs[3 * r + 0], ny = dirs[3 * r + 1], nz = dirs[3 * r + 2];
        if (nz == 0.0) return -1;
        const double sigma = nz > 0.0 ? 1.0 : -1.0;
        const uint8_t upwall = nz > 0.0 ? 1 : 2;
        int64_t nfb = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int64_t o = (int64_t)r * n + i;
            k1[o] = -1; k2[o] = -1; w1[o] = 1.0; ds1[o] = 0.0; ds2[o] = 0.0;
            if (wall[i] & upwall) continue; /* boundary site (R4) */
            orc_cand best1 = {-1, -1, 0.0, 0.0, 1.0}, best2 = best1, fb = best1;
            int nc = 0, nfbc = 0;
            for (int64_t e = nbr_ptr[i]; e < nbr_ptr[i + 1]; ++e) {
                const int32_t k = nbr_idx[e];
                const double dx = (xyz[3 * i + 0] - xyz[3 * k + 0]) - (double)nbr_shift[2 * e + 0] * Lx;
                const double dy = (xyz[3 * i + 1] - xyz[3 * k + 1]) - (double)nbr_shift[2 * e + 1] * Ly;
                const double dz = xyz[3 * i + 2] - xyz[3 * k + 2];
                if (!(sigma * dz > 0.0)) continue; /* not strictly upwind in height */
                orc_cand c;
                c.k = k; c.e = e;
                c.dot = nx * dx + ny * dy + nz * dz;
                c.len2 = dx * dx + dy * dy + dz * dz;
                c.q = (c.dot * fabs(c.dot)) / c.len2;
                if (nfbc == 0 || orc_before(&c, &fb)) fb = c;
                nfbc++;
                if (c.dot > 0.0) {
                    if (nc == 0) best1 = c;
                    else if (orc_before(&c, &best1)) { best2 = best1; best1 = c; }
                    else if (nc == 1 || orc_before(&c, &best2)) best2 = c;
                    nc++;
                }
            }
            if (nc >= 2) {
                const double v1 = best1.dot / sqrt(best1.len2);
                const double v2 = best2.dot / sqrt(best2.len2);
                const double a = pow(v1, r_exp), b = pow(v2, r_exp);
                k1[o] = best1.k; k2[o] = best2.k;
                w1[o] = a / (a + b);
                ds1[o] = sqrt(best1.len2); ds2[o] = sqrt(best2.len2);
            } else if (nc == 1) {
                k1[o] = best1.k; ds1[o] = sqrt(best1.len2);
            } else if (nfbc > 0) {
                k1[o] = fb.k; ds1[o] = sqrt(fb.len2); nfb++;
            } else {
                status = -2;
            }
        }
        if (n_fallback) n_fallback[r] = nfb;
    }
    return status;
}

/* ---------------------------------------------------------------------------
 * Level schedule of one ray's upwind graph (Sect. 2.5: sweeps start at the
 * upwind boundary). level = 0 for boundary sites, else 1 + the largest level
 * of the chosen upwind sites. order = sites sorted by (level, index);
 * level_ptr[l] = first position of level l. Computed by one pass in height
 * order (every dependency is strictly upwind in z).
 * ------------------------------------------------------------------------- */
static const double *g_sort_z;
static double g_sort_sigma;
static int orc_cmp_z(const void *pa, const void *pb) {
    const int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    const double za = g_sort_sigma * g_sort_z[3 * a + 2], zb = g_sort_sigma * g_sort_z[3 * b + 2];
    if (za < zb) return -1;
    if (za > zb) return 1;
    return (a > b) - (a < b);
}

/* sweep order of one ray: sites sorted by (sigma*z, index); not thread-safe */
void orc_height_order(int64_t n, const double *xyz, double sigma, int64_t *out) {
    for (int64_t i = 0; i < n; ++i) out[i] = i;
    g_sort_z = xyz;
    g_sort_sigma = sigma;
    qsort(out, (size_t)n, sizeof(int64_t), orc_cmp_z);
}

int orc_levels(int64_t n, const double *xyz, int32_t n_rays, const double *dirs, const int32_t *k1,
               const int32_t *k2, int32_t *level, int32_t *order, int32_t *level_ptr /* [R][n+1] */,
               int32_t *n_levels) {
    int64_t *hz = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *cnt = (int64_t *)calloc((size_t)n + 2, sizeof(int64_t));
    if (!hz || !cnt) { free(hz); free(cnt); return -5; }
    for (int32_t r = 0; r < n_rays; ++r) {
        const double sigma = dirs[3 * r + 2] > 0.0 ? 1.0 : -1.0;
        const int32_t *K1 = k1 + (int64_t)r * n, *K2 = k2 + (int64_t)r * n;
        int32_t *lev = level + (int64_t)r * n;
        orc_height_order(n, xyz, sigma, hz);
        int32_t lmax = -1;
        for (int64_t p = 0; p < n; ++p) {
            const int64_t i = hz[p];
            int32_t l = 0;
            if (K1[i] >= 0) {
                l = lev[K1[i]];
                if (K2[i] >= 0 && lev[K2[i]] > l) l = lev[K2[i]];
                l += 1;
            }
            lev[i] = l;
            if (l > lmax) lmax = l;
        }
        const int32_t L = lmax + 1;
        n_levels[r] = L;
        memset(cnt, 0, sizeof(int64_t) * ((size_t)n + 2));
        for (int64_t i = 0; i < n; ++i) cnt[lev[i] + 1]++;
        for (int32_t l = 0; l < L; ++l) cnt[l + 1] += cnt[l];
        int32_t *lp = level_ptr + (int64_t)r * (n + 1);
        for (int32_t l = 0; l <= L; ++l) lp[l] = (int32_t)cnt[l];
        int32_t *ord = order + (int64_t)r * n;
        for (int64_t i = 0; i < n; ++i) ord[cnt[lev[i]]++] = (int32_t)i;
    }
    free(hz);
    free(cnt);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Formal solution on the Voronoi grid for every ray and wavelength, and the
 * mean intensity J = sum_r w_r I_r (Eq. 2, 4, 5).
 * chi, S, I_bottom, I_top are [n][nl]; I_top may be NULL (= 0). I_out, if not
 * NULL, receives [R][n][nl]. J receives [n][nl]. Rays are processed in groups
 * of one per thread; J is accumulated in ray order so the result does not
 * depend on the thread count.
 * ------------------------------------------------------------------------- */
static void orc_sweep_one_ray(int64_t n, int32_t nl, double nz, const int32_t *K1,
                              const int32_t *K2, const double *W1, const double *D1, const double *D2,
                              const double *chi, const double *S, const double *Ibot, const double *Itop,
                              const int64_t *hz, double *I) {
    for (int64_t p = 0; p < n; ++p) {
        const int64_t i = hz[p];
        double *Ii = I + i * nl;
        if (K1[i] < 0) {
            for (int32_t l = 0; l < nl; ++l)
                Ii[l] = nz > 0.0 ? Ibot[i * nl + l] : (Itop ? Itop[i * nl + l] : 0.0);
            continue;
        }
        const int64_t ka = K1[i], kb = K2[i];
        for (int32_t l = 0; l < nl; ++l) {
            const double chi_i = chi[i * nl + l], S_i = S[i * nl + l];
            double E, pu, p0;
            const double xa = 0.5 * (chi[ka * nl + l] + chi_i) * D1[i];
            orc_psi(xa, &E, &pu, &p0);
            const double Ia = E * I[ka * nl + l] + pu * S[ka * nl + l] + p0 * S_i;
            if (kb >= 0) {
                const double xb = 0.5 * (chi[kb * nl + l] + chi_i) * D2[i];
                orc_psi(xb, &E, &pu, &p0);
                const double Ib = E * I[kb * nl + l] + pu * S[kb * nl + l] + p0 * S_i;
                Ii[l] = W1[i] * Ia + (1.0 - W1[i]) * Ib;
            } else {
                Ii[l] = Ia;
            }
        }
    }
}

int orc_fs_voronoi(int64_t n, int32_t n_rays, int32_t nl, const double *xyz, const double *dirs,
                   const double *ray_w, const int32_t *k1, const int32_t *k2, const double *w1,
                   const double *ds1, const double *ds2, const double *chi, const double *S,
                   const double *I_bottom, const double *I_top, double *I_out, double *J) {
    const int64_t nn = n * (int64_t)nl;
    int nth = orc_num_threads();
    if (nth > n_rays) nth = n_rays;
    if (nth < 1) nth = 1;
    double *buf = NULL;
    if (!I_out) {
        buf = (double *)malloc(sizeof(double) * (size_t)nth * (size_t)(nn > 0 ? nn : 1));
        if (!buf) return -5;
    }
    /* sweep orders for upward (ascending z) and downward (descending z) rays,
     * computed once, serially: the sort helper keeps its key in file-scope state */
    int64_t *hz = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)(n > 0 ? n : 1));
    if (!hz) { free(buf); return -5; }
    orc_height_order(n, xyz, 1.0, hz);
    orc_height_order(n, xyz, -1.0, hz + n);
    for (int64_t t = 0; t < nn; ++t) J[t] = 0.0;
    for (int32_t r0 = 0; r0 < n_rays; r0 += nth) {
        const int32_t cnt = (n_rays - r0) < nth ? (n_rays - r0) : nth;
#pragma omp parallel for schedule(static, 1) num_threads(nth)
        for (int32_t t = 0; t < cnt; ++t) {
            const int32_t r = r0 + t;
            double *I = I_out ? I_out + (int64_t)r * nn : buf + (int64_t)t * nn;
            orc_sweep_one_ray(n, nl, dirs[3 * r + 2], k1 + (int64_t)r * n, k2 + (int64_t)r * n,
                              w1 + (int64_t)r * n, ds1 + (int64_t)r * n, ds2 + (int64_t)r * n, chi, S,
                              I_bottom, I_top, dirs[3 * r + 2] > 0.0 ? hz : hz + n, I);
        }
        for (int32_t t = 0; t < cnt; ++t) {
            const int32_t r = r0 + t;
            const double *I = I_out ? I_out + (int64_t)r * nn : buf + (int64_t)t * nn;
            for (int64_t q = 0; q < nn; ++q) J[q] += ray_w[r] * I[q];
        }
    }
    free(buf);
    free(hz);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Short characteristics on a regular grid (Sect. 2.6; reading R6).
 * Fields are [z][y][x][nl]; x_i = i dx, y_j = j dy, periodic in x and y with
 * periods nx dx and ny dy; z is strictly increasing. Plane 0 takes I_bottom
 * on upward rays; the top plane takes I_top (NULL = 0) on downward rays.
 * ------------------------------------------------------------------------- */
static void orc_bilinear_weights(double xq, double d, int32_t nper, int32_t *i0, int32_t *i1, double *t) {
    const double f = xq / d;
    const double fl = floor(f);
    *t = f - fl;
    int64_t a = (int64_t)fl % nper;
    if (a < 0) a += nper;
    *i0 = (int32_t)a;
    *i1 = (int32_t)((a + 1) % nper);
}

int orc_fs_regular(int32_t nx, int32_t ny, int32_t nz, double dx, double dy, const double *z, int32_t n_rays,
                   const double *dirs, const double *ray_w, int32_t nl, const double *chi, const double *S,
                   const double *I_bottom, const double *I_top, double *I_out, double *J) {
    const int64_t plane = (int64_t)nx * ny;
    const int64_t n = plane * nz;
    const int64_t nn = n * nl;
    int nth = orc_num_threads();
    if (nth > n_rays) nth = n_rays;
    if (nth < 1) nth = 1;
    double *buf = NULL;
    if (!I_out) {
        buf = (double *)malloc(sizeof(double) * (size_t)nth * (size_t)(nn > 0 ? nn : 1));
        if (!buf) return -5;
    }
    for (int64_t t = 0; t < nn; ++t) J[t] = 0.0;
    for (int32_t r0 = 0; r0 < n_rays; r0 += nth) {
        const int32_t cnt = (n_rays - r0) < nth ? (n_rays - r0) : nth;
#pragma omp parallel for schedule(static, 1) num_threads(nth)
        for (int32_t t = 0; t < cnt; ++t) {
            const int32_t r = r0 + t;
            double *I = I_out ? I_out + (int64_t)r * nn : buf + (int64_t)t * nn;
            const double mx = dirs[3 * r + 0], my = dirs[3 * r + 1], mz = dirs[3 * r + 2];
            const int up = mz > 0.0;
            for (int32_t s = 0; s < nz; ++s) {
                const int32_t k = up ? s : nz - 1 - s;
                if (s == 0) {
                    for (int64_t q = 0; q < plane * nl; ++q) {
                        const int64_t g = (int64_t)k * plane * nl + q;
                        I[g] = up ? I_bottom[g] : (I_top ? I_top[g] : 0.0);
                    }
                    continue;
                }
                const int32_t ku = up ? k - 1 : k + 1; /* upwind plane */
                const double dz = fabs(z[k] - z[ku]);
                const double ds = dz / fabs(mz);
                for (int32_t j = 0; j < ny; ++j) {
                    for (int32_t i = 0; i < nx; ++i) {
                        int32_t ix0, ix1, iy0, iy1;
                        double tx, ty;
                        orc_bilinear_weights((double)i * dx - ds * mx, dx, nx, &ix0, &ix1, &tx);
                        orc_bilinear_weights((double)j * dy - ds * my, dy, ny, &iy0, &iy1, &ty);
                        const int64_t c00 = ((int64_t)ku * ny + iy0) * nx + ix0;
                        const int64_t c10 = ((int64_t)ku * ny + iy0) * nx + ix1;
                        const int64_t c01 = ((int64_t)ku * ny + iy1) * nx + ix0;
                        const int64_t c11 = ((int64_t)ku * ny + iy1) * nx + ix1;
                        const double a00 = (1.0 - tx) * (1.0 - ty), a10 = tx * (1.0 - ty);
                        const double a01 = (1.0 - tx) * ty, a11 = tx * ty;
                        const int64_t me = ((int64_t)k * ny + j) * nx + i;
                        for (int32_t l = 0; l < nl; ++l) {
                            const double Iu = a00 * I[c00 * nl + l] + a10 * I[c10 * nl + l] +
                                              a01 * I[c01 * nl + l] + a11 * I[c11 * nl + l];
                            const double Su = a00 * S[c00 * nl + l] + a10 * S[c10 * nl + l] +
                                              a01 * S[c01 * nl + l] + a11 * S[c11 * nl + l];
                            const double cu = a00 * chi[c00 * nl + l] + a10 * chi[c10 * nl + l] +
                                              a01 * chi[c01 * nl + l] + a11 * chi[c11 * nl + l];
                            const double x = 0.5 * (cu + chi[me * nl + l]) * ds;
                            double E, pu, p0;
                            orc_psi(x, &E, &pu, &p0);
                            I[me * nl + l] = E * Iu + pu * Su + p0 * S[me * nl + l];
                        }
                    }
                }
            }
        }
        for (int32_t t = 0; t < cnt; ++t) {
            const int32_t r = r0 + t;
            const double *I = I_out ? I_out + (int64_t)r * nn : buf + (int64_t)t * nn;
            for (int64_t q = 0; q < nn; ++q) J[q] += ray_w[r] * I[q];
        }
    }
    free(buf);
    return 0;
}

/* ---------------------------------------------------------------------------
 * LTE grey continuum (Sect. 2.1 with S = B): chi = kappa0 rho^2 T^9 at every
 * wavelength (kappa0 rho T^9 is a mass absorption coefficient), S = B_lambda(T)
 * and the thermalised lower boundary I_bottom = B_lambda(T).
 * Planck function in kW m^-2 nm^-1 sr^-1: B = 2 h c^2 / lambda^5 / (e^u - 1),
 * u = h c / (lambda k T), times 1e-12 to convert W m^-2 m^-1 to kW m^-2 nm^-1.
 * ------------------------------------------------------------------------- */
static const double ORC_H = 6.62607015e-34;  /* J s (exact, SI 2019) */
static const double ORC_C = 299792458.0;     /* m / s (exact) */
static const double ORC_K = 1.380649e-23;    /* J / K (exact, SI 2019) */

double orc_planck(double lam, double T) {
    const double u = ORC_H * ORC_C / (lam * ORC_K * T);
    return 2.0 * ORC_H * ORC_C * ORC_C / pow(lam, 5.0) / expm1(u) * 1e-12;
}

/* dB/dT at fixed wavelength */
double orc_dplanck_dT(double lam, double T) {
    const double u = ORC_H * ORC_C / (lam * ORC_K * T);
    const double B = orc_planck(lam, T);
    return B * (u / T) * exp(u) / expm1(u);
}

void orc_lte(int64_t n, int32_t nl, const double *lam, double kappa0, const double *T, const double *rho,
             double *chi, double *S) {
    for (int64_t i = 0; i < n; ++i) {
        const double c = kappa0 * rho[i] * rho[i] * pow(T[i], 9.0);
        for (int32_t l = 0; l < nl; ++l) {
            chi[i * nl + l] = c;
            S[i * nl + l] = orc_planck(lam[l], T[i]);
        }
    }
}

/* ---------------------------------------------------------------------------
 * Reverse (adjoint) sweep of the Voronoi formal solution: given dL/dI for
 * every ray, site and wavelength (dL_dI, [R][n][nl], may be NULL) and dL/dJ
 * ([n][nl], may be NULL; J = sum_r w_r I_r), accumulate dL/dchi, dL/dS,
 * dL/dI_bottom and dL/dI_top ([n][nl] each, overwritten). I is the forward
 * intensity [R][n][nl]. Written in scatter form: sites are visited in the
 * exact reverse of the forward sweep order, and each site's adjoint is pushed
 * to the quantities its forward update read:
 *   I_i = sum_j w_j (E_j I_kj + Psi_u,j S_kj + Psi_0,j S_i),
 *   x_j = (chi_kj + chi_i) ds_j / 2.
 * ------------------------------------------------------------------------- */
int orc_fs_voronoi_vjp(int64_t n, int32_t n_rays, int32_t nl, const double *xyz, const double *dirs,
                       const double *ray_w, const int32_t *k1, const int32_t *k2, const double *w1,
                       const double *ds1, const double *ds2, const double *chi, const double *S, const double *I,
                       const double *dL_dI, const double *dL_dJ, double *g_chi, double *g_S, double *g_Ib,
                       double *g_It) {
    const int64_t nn = n * (int64_t)nl;
    for (int64_t q = 0; q < nn; ++q) { g_chi[q] = 0.0; g_S[q] = 0.0; g_Ib[q] = 0.0; g_It[q] = 0.0; }
    double *Ibar = (double *)malloc(sizeof(double) * (size_t)(nn > 0 ? nn : 1));
    int64_t *hz = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!Ibar || !hz) { free(Ibar); free(hz); return -5; }
    for (int32_t r = 0; r < n_rays; ++r) {
        const double nz = dirs[3 * r + 2];
        const int32_t *K1 = k1 + (int64_t)r * n, *K2 = k2 + (int64_t)r * n;
        const double *W1 = w1 + (int64_t)r * n, *D1 = ds1 + (int64_t)r * n, *D2 = ds2 + (int64_t)r * n;
        const double *Ir = I + (int64_t)r * nn;
        for (int64_t q = 0; q < nn; ++q) {
            Ibar[q] = dL_dI ? dL_dI[(int64_t)r * nn + q] : 0.0;
            if (dL_dJ) Ibar[q] += ray_w[r] * dL_dJ[q];
        }
        orc_height_order(n, xyz, nz > 0.0 ? 1.0 : -1.0, hz);
        /* wavelengths never mix: each thread takes a contiguous range of them and
         * walks the sites in the same order, so every sum is formed in the same
         * order as by a single thread */
        const int nth = orc_num_threads();
        const int32_t chunks = nl < nth ? nl : nth;
#pragma omp parallel for schedule(static, 1) num_threads(nth)
        for (int32_t c = 0; c < chunks; ++c) {
          const int32_t l0 = (int32_t)((int64_t)c * nl / chunks), l1 = (int32_t)((int64_t)(c + 1) * nl / chunks);
          for (int64_t p = n - 1; p >= 0; --p) {
            const int64_t i = hz[p];
            if (K1[i] < 0) {
                double *gb = nz > 0.0 ? g_Ib : g_It;
                for (int32_t l = l0; l < l1; ++l) gb[i * nl + l] += Ibar[i * nl + l];
                continue;
            }
            for (int j = 0; j < 2; ++j) {
                const int64_t k = j == 0 ? K1[i] : K2[i];
                if (k < 0) continue;
                const double w = (K2[i] < 0) ? 1.0 : (j == 0 ? W1[i] : 1.0 - W1[i]);
                const double ds = j == 0 ? D1[i] : D2[i];
                for (int32_t l = l0; l < l1; ++l) {
                    const double gi = Ibar[i * nl + l] * w;
                    if (gi == 0.0) continue;
                    const double x = 0.5 * (chi[k * nl + l] + chi[i * nl + l]) * ds;
                    double E, pu, p0, dpu, dp0;
                    orc_psi(x, &E, &pu, &p0);
                    orc_dpsi(x, &dpu, &dp0);
                    Ibar[k * nl + l] += gi * E;
                    g_S[k * nl + l] += gi * pu;
                    g_S[i * nl + l] += gi * p0;
                    const double xbar = gi * (-E * Ir[k * nl + l] + dpu * S[k * nl + l] + dp0 * S[i * nl + l]);
                    g_chi[k * nl + l] += 0.5 * ds * xbar;
                    g_chi[i * nl + l] += 0.5 * ds * xbar;
                }
            }
          }
        }
    }
    free(Ibar);
    free(hz);
    return 0;
}

/* Chain rule of the grey LTE continuum to temperature and density:
 *   chi = kappa0 rho^2 T^9  ->  dchi/dT = 9 chi / T,  dchi/drho = 2 chi / rho,
 *   S = I_bottom = B_lambda(T) ->  dB/dT.
 * g_T, g_rho [n] receive sum over wavelengths. */
void orc_lte_vjp(int64_t n, int32_t nl, const double *lam, double kappa0, const double *T, const double *rho,
                 const double *g_chi, const double *g_S, const double *g_Ib, double *g_T, double *g_rho) {
    for (int64_t i = 0; i < n; ++i) {
        const double c = kappa0 * rho[i] * rho[i] * pow(T[i], 9.0);
        double gt = 0.0, gr = 0.0;
        for (int32_t l = 0; l < nl; ++l) {
            const int64_t q = i * nl + l;
            gt += g_chi[q] * 9.0 * c / T[i] + (g_S[q] + (g_Ib ? g_Ib[q] : 0.0)) * orc_dplanck_dT(lam[l], T[i]);
            gr += g_chi[q] * 2.0 * c / rho[i];
        }
        g_T[i] = gt;
        g_rho[i] = gr;
    }
}

/* ---------------------------------------------------------------------------
 * Local (diagonal) operator of the formal solution, for the accelerated
 * Lambda iteration (the Jacobi operator the paper names as the cure for small
 * eps, Sect. 2.2): along ray r, site i's intensity depends on its own source
 * function only through the Psi_0 S_i term of each of its upwind lines
 * (Eq. 2 with linear S, Eq. 5), and the upwind intensities never depend on
 * S_i. Hence
 *   Lambda*_ii = dJ_i/dS_i = sum_r w_r sum_j w_j Psi_0(x_j),
 * with x_j = (chi_kj + chi_i) ds_j / 2, w_j the Eq. 5 weights (1 for a single
 * line) and 0 at a ray's upwind-boundary sites. out [n][nl].
 * ------------------------------------------------------------------------- */
void orc_lambda_diag(int64_t n, int32_t n_rays, int32_t nl, const double *ray_w, const int32_t *k1,
                     const int32_t *k2, const double *w1, const double *ds1, const double *ds2,
                     const double *chi, double *out) {
    for (int64_t q = 0; q < n * (int64_t)nl; ++q) out[q] = 0.0;
    for (int32_t r = 0; r < n_rays; ++r) {
        for (int64_t i = 0; i < n; ++i) {
            const int64_t ri = (int64_t)r * n + i;
            if (k1[ri] < 0) continue;
            for (int32_t l = 0; l < nl; ++l) {
                double E, pu, p0, sum = 0.0;
                const double ci = chi[i * nl + l];
                if (k2[ri] < 0) {
                    orc_psi(0.5 * (chi[(int64_t)k1[ri] * nl + l] + ci) * ds1[ri], &E, &pu, &p0);
                    sum = p0;
                } else {
                    orc_psi(0.5 * (chi[(int64_t)k1[ri] * nl + l] + ci) * ds1[ri], &E, &pu, &p0);
                    sum = w1[ri] * p0;
                    orc_psi(0.5 * (chi[(int64_t)k2[ri] * nl + l] + ci) * ds2[ri], &E, &pu, &p0);
                    sum += (1.0 - w1[ri]) * p0;
                }
                out[i * nl + l] += ray_w[r] * sum;
            }
        }
    }
}

/* ---------------------------------------------------------------------------
 * Final synthesis (Sect. 2.5, closing paragraph; Sect. 3.2): the converged
 * solution on the irregular grid is carried back to a regular grid by
 * inverse-distance interpolation from the two nearest sites, and the emergent
 * intensity at mu = 1 is then a long-characteristics solution along each
 * vertical column of that grid.
 *
 * orc_idw2: for every query point q, the two distinct sites nearest to it,
 * found by brute force over all sites. Distance (reading S1): components
 * dx = xq - xs and dy = yq - ys are brought into [-L/2, L/2] by adding or
 * subtracting the period L when the grid is periodic in x and y, dz = zq - zs,
 * and d2 = dx*dx + dy*dy + dz*dz in that order (no fused multiply-add). Keys
 * (d2, site index) are compared lexicographically, so ties go to the smaller
 * index. Weights (reading S2): u_k = d_k^-p, w1 = u_1 / (u_1 + u_2), written
 * as w1 = a_2 / (a_1 + a_2) with a_k = d_k^p = (d2_k)^(p/2), which is 1 when
 * d_1 = 0; w1 = 1 when both distances are 0. A grid with one site gives
 * i2 = i1 and w1 = 1. Outputs idx [m][2], w1 [m], d2 [m][2] (d2 may be NULL).
 * ------------------------------------------------------------------------- */
static double orc_wrap(double d, int periodic, double L) {
    if (!periodic) return d;
    const double h = 0.5 * L;
    while (d > h) d -= L;
    while (d < -h) d += L;
    return d;
}

void orc_idw2(int64_t n, const double *xyz, int64_t m, const double *pts, int periodic, double Lx, double Ly,
              double power, int32_t *idx, double *w1, double *d2out) {
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < m; ++q) {
        int64_t b1 = -1, b2 = -1;
        double e1 = 0.0, e2 = 0.0;
        for (int64_t s = 0; s < n; ++s) {
            const double dx = orc_wrap(pts[3 * q + 0] - xyz[3 * s + 0], periodic, Lx);
            const double dy = orc_wrap(pts[3 * q + 1] - xyz[3 * s + 1], periodic, Ly);
            const double dz = pts[3 * q + 2] - xyz[3 * s + 2];
            const double d2 = dx * dx + dy * dy + dz * dz;
            /* sites arrive in increasing index, so a strict < keeps the smaller index on ties */
            if (b1 < 0 || d2 < e1) {
                b2 = b1;
                e2 = e1;
                b1 = s;
                e1 = d2;
            } else if (b2 < 0 || d2 < e2) {
                b2 = s;
                e2 = d2;
            }
        }
        double w = 1.0;
        if (b2 < 0) {
            b2 = b1;
            e2 = e1;
        } else {
            const double a1 = pow(e1, 0.5 * power), a2 = pow(e2, 0.5 * power);
            if (a1 + a2 > 0.0) w = a2 / (a1 + a2);
        }
        idx[2 * q + 0] = (int32_t)b1;
        idx[2 * q + 1] = (int32_t)b2;
        w1[q] = w;
        if (d2out) {
            d2out[2 * q + 0] = e1;
            d2out[2 * q + 1] = e2;
        }
    }
}

/* ---------------------------------------------------------------------------
 * Long characteristics at mu = 1 (Sect. 2.5, closing paragraph): along each
 * vertical column c of a regular grid, from the bottom plane upwards,
 *   I_0 = I_bottom[c],  I_k = e^-x I_(k-1) + Psi_u(x) S_(k-1) + Psi_0(x) S_k,
 *   x = (chi_(k-1) + chi_k) / 2 * (z_k - z_(k-1)),
 * the linear-source step of Eq. 2 with the trapezoid optical depth (R5). The
 * result is I at the top plane. chi, S [nz * ncol][nl] (point (k, c) at row
 * k * ncol + c), I_bottom and I_top [ncol][nl].
 * ------------------------------------------------------------------------- */
void orc_lc_vertical(int64_t ncol, int32_t nz, int32_t nl, const double *z, const double *chi, const double *S,
                     const double *I_bottom, double *I_top) {
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncol; ++c) {
        for (int32_t l = 0; l < nl; ++l) {
            double I = I_bottom[c * nl + l];
            for (int32_t k = 1; k < nz; ++k) {
                const int64_t lo = ((int64_t)(k - 1) * ncol + c) * nl + l;
                const int64_t hi = ((int64_t)k * ncol + c) * nl + l;
                const double x = 0.5 * (chi[lo] + chi[hi]) * (z[k] - z[k - 1]);
                double E, pu, p0;
                orc_psi(x, &E, &pu, &p0);
                I = E * I + pu * S[lo] + p0 * S[hi];
            }
            I_top[c * nl + l] = I;
        }
    }
}

/* ---------------------------------------------------------------------------
 * Quadratic Bezier segment (the higher-order scheme the paper points to in
 * Sect. 2.5: de la Cruz Rodriguez & Piskunov 2013). Along a segment of
 * optical depth x from an upwind point u to the point 0, S is the quadratic
 * Bezier curve with end values S_u, S_0 and control value C; with s = t/x,
 *   S(t) = S_u (1 - s)^2 + 2 C s (1 - s) + S_0 s^2,
 *   I_0 = e^-x I_u + alpha S_u + beta S_0 + gamma C,
 *   alpha = int_0^x (1-s)^2 e^-(x-t) dt = [2 - e^-x (x^2 + 2x + 2)] / x^2,
 *   beta  = int_0^x s^2 e^-(x-t) dt     = 1 - 2 (e^-x + x - 1) / x^2,
 *   gamma = int_0^x 2s(1-s) e^-(x-t) dt = 2 (x - 2 + e^-x (x + 2)) / x^2.
 * Below x = 1 the three are summed from their power series,
 *   alpha = sum_{m>=3} (-1)^(m+1) (m-1)(m-2) x^(m-2) / m!,
 *   beta  = sum_{m>=3} 2 (-1)^(m+1) x^(m-2) / m!,
 *   gamma = sum_{m>=3} 2 (-1)^(m+1) (m-2) x^(m-2) / m!,
 * which removes the cancellation of the closed forms at small x.
 * ------------------------------------------------------------------------- */
void orc_bezier_weights(double x, double *E, double *alpha, double *beta, double *gamma) {
    const double e = exp(-x);
    *E = e;
    if (x < 1.0) {
        double a = 0.0, b = 0.0, c = 0.0;
        double p = x / 6.0; /* x^(m-2)/m! for m = 3 */
        for (int m = 3; m <= 45; ++m) {
            const double sg = (m % 2 == 1) ? 1.0 : -1.0; /* (-1)^(m+1) */
            a += sg * (double)((m - 1) * (m - 2)) * p;
            b += sg * 2.0 * p;
            c += sg * 2.0 * (double)(m - 2) * p;
            p *= x / (double)(m + 1);
        }
        *alpha = a;
        *beta = b;
        *gamma = c;
    } else {
        const double x2 = x * x;
        *alpha = (2.0 - e * (x2 + 2.0 * x + 2.0)) / x2;
        *beta = 1.0 - 2.0 * (e + x - 1.0) / x2;
        *gamma = 2.0 * (x - 2.0 + e * (x + 2.0)) / x2;
    }
}

/* Control value of one upwind line (reading Q1). The derivative of S at the
 * point 0 along the ray comes from the upwind slope d_u = (S_0 - S_u)/x and
 * the downwind slope d_d (weighted over the downwind lines, of optical depth
 * x_d) by the Fritsch-Butland harmonic mean:
 *   S' = d_u d_d / (a d_d + (1 - a) d_u),  a = (1 + x_d / (x + x_d)) / 3,
 * when d_u d_d > 0, else S' = 0; without downwind lines S' = d_u (the
 * segment is then linear). C = S_0 - x S' / 2, kept between S_u and S_0.
 * has_d: whether downwind data exist (x_d > 0). */
static double orc_bezier_control(double Su, double S0, double x, int has_d, double dd, double xd) {
    if (!(x > 0.0)) return S0;
    const double du = (S0 - Su) / x;
    double d;
    if (!has_d) {
        d = du;
    } else if (du * dd > 0.0) {
        const double a = (1.0 + xd / (x + xd)) / 3.0;
        d = du * dd / (a * dd + (1.0 - a) * du);
    } else {
        d = 0.0;
    }
    double C = S0 - 0.5 * x * d;
    const double lo = Su < S0 ? Su : S0, hi = Su < S0 ? S0 : Su;
    if (C < lo) C = lo;
    if (C > hi) C = hi;
    return C;
}

/* ---------------------------------------------------------------------------
 * Voronoi formal solution with the quadratic Bezier segment (reading Q1).
 * As orc_fs_voronoi, plus the downwind lines of every (ray, site): the upwind
 * selection of the opposite direction (q1, q2 sites, qw1 weight of q1, qd1,
 * qd2 lengths; q1 < 0 at sites on the far wall). For site i, wavelength l:
 *   x'_j = (chi_qj + chi_i)/2 qd_j,  d_d = sum_j qw_j (S_qj - S_i)/x'_j,
 *   x_d = sum_j qw_j x'_j  (qw_2 = 1 - qw1; one line: weight 1);
 * every upwind line j then gives I_j = e^-x I_kj + alpha S_kj + beta S_i +
 * gamma C_j with C_j from orc_bezier_control, and I_i = sum_j w_j I_j (Eq. 5).
 * A zero downwind optical depth leaves the downwind slope unused.
 * ------------------------------------------------------------------------- */
static void orc_sweep_one_ray_bezier(int64_t n, int32_t nl, double nz, const int32_t *K1, const int32_t *K2,
                                     const double *W1, const double *D1, const double *D2, const int32_t *Q1,
                                     const int32_t *Q2, const double *QW1, const double *QD1, const double *QD2,
                                     const double *chi, const double *S, const double *Ibot, const double *Itop,
                                     const int64_t *hz, double *I) {
    for (int64_t p = 0; p < n; ++p) {
        const int64_t i = hz[p];
        double *Ii = I + i * nl;
        if (K1[i] < 0) {
            for (int32_t l = 0; l < nl; ++l)
                Ii[l] = nz > 0.0 ? Ibot[i * nl + l] : (Itop ? Itop[i * nl + l] : 0.0);
            continue;
        }
        for (int32_t l = 0; l < nl; ++l) {
            const double chi_i = chi[i * nl + l], S_i = S[i * nl + l];
            /* downwind slope and optical depth */
            int has_d = Q1[i] >= 0;
            double dd = 0.0, xd = 0.0;
            if (has_d) {
                const int nq = Q2[i] >= 0 ? 2 : 1;
                for (int j = 0; j < nq; ++j) {
                    const int64_t q = j == 0 ? Q1[i] : Q2[i];
                    const double wq = nq == 1 ? 1.0 : (j == 0 ? QW1[i] : 1.0 - QW1[i]);
                    const double xq = 0.5 * (chi[q * nl + l] + chi_i) * (j == 0 ? QD1[i] : QD2[i]);
                    if (!(xq > 0.0)) {
                        has_d = 0;
                        break;
                    }
                    dd += wq * (S[q * nl + l] - S_i) / xq;
                    xd += wq * xq;
                }
            }
            const int nk = K2[i] >= 0 ? 2 : 1;
            double sum = 0.0;
            for (int j = 0; j < nk; ++j) {
                const int64_t k = j == 0 ? K1[i] : K2[i];
                const double w = nk == 1 ? 1.0 : (j == 0 ? W1[i] : 1.0 - W1[i]);
                const double x = 0.5 * (chi[k * nl + l] + chi_i) * (j == 0 ? D1[i] : D2[i]);
                const double Su = S[k * nl + l];
                const double C = orc_bezier_control(Su, S_i, x, has_d, dd, xd);
                double E, a, b, c;
                orc_bezier_weights(x, &E, &a, &b, &c);
                sum += w * (E * I[k * nl + l] + a * Su + b * S_i + c * C);
            }
            Ii[l] = sum;
        }
    }
}

int orc_fs_voronoi_bezier(int64_t n, int32_t n_rays, int32_t nl, const double *xyz, const double *dirs,
                          const double *ray_w, const int32_t *k1, const int32_t *k2, const double *w1,
                          const double *ds1, const double *ds2, const int32_t *q1, const int32_t *q2,
                          const double *qw1, const double *qd1, const double *qd2, const double *chi, const double *S,
                          const double *I_bottom, const double *I_top, double *I_out, double *J) {
    const int64_t nn = n * (int64_t)nl;
    int nth = orc_num_threads();
    if (nth > n_rays) nth = n_rays;
    if (nth < 1) nth = 1;
    double *buf = NULL;
    if (!I_out) {
        buf = (double *)malloc(sizeof(double) * (size_t)nth * (size_t)(nn > 0 ? nn : 1));
        if (!buf) return -5;
    }
    int64_t *hz = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)(n > 0 ? n : 1));
    if (!hz) { free(buf); return -5; }
    orc_height_order(n, xyz, 1.0, hz);
    orc_height_order(n, xyz, -1.0, hz + n);
    for (int64_t t = 0; t < nn; ++t) J[t] = 0.0;
    for (int32_t r0 = 0; r0 < n_rays; r0 += nth) {
        const int32_t cnt = (n_rays - r0) < nth ? (n_rays - r0) : nth;
#pragma omp parallel for schedule(static, 1) num_threads(nth)
        for (int32_t t = 0; t < cnt; ++t) {
            const int32_t r = r0 + t;
            const int64_t o = (int64_t)r * n;
            double *I = I_out ? I_out + (int64_t)r * nn : buf + (int64_t)t * nn;
            orc_sweep_one_ray_bezier(n, nl, dirs[3 * r + 2], k1 + o, k2 + o, w1 + o, ds1 + o, ds2 + o, q1 + o, q2 + o,
                                     qw1 + o, qd1 + o, qd2 + o, chi, S, I_bottom, I_top,
                                     dirs[3 * r + 2] > 0.0 ? hz : hz + n, I);
        }
        for (int32_t t = 0; t < cnt; ++t) {
            const int32_t r = r0 + t;
            const double *I = I_out ? I_out + (int64_t)r * nn : buf + (int64_t)t * nn;
            for (int64_t q = 0; q < nn; ++q) J[q] += ray_w[r] * I[q];
        }
    }
    free(buf);
    free(hz);
    return 0;
}
