/*
 * vrt.h -- C ABI of the MI355X (gfx950) formal-solution library.
 *
 * The library solves the time-independent radiative transfer equation
 * dI/dtau = S - I along every ray of a fixed angle quadrature, on an
 * irregular (Voronoi) grid or on a regular grid, and integrates the
 * intensities over angle to the mean intensity J (Udnaes & Pereira 2023,
 * Sect. 2.1, Eq. 1, 2 and 4). On a Voronoi grid the intensity at a site is
 * carried along the two Delaunay lines closest to the ray direction and
 * weighted by w_j = v_j^r / (v_1^r + v_2^r) (Sect. 2.5, Eq. 5 and 6); along
 * each line the source function is taken as linear (Sect. 2.5). On a regular
 * grid short characteristics with bilinear interpolation in the upwind
 * horizontal plane are used (Sect. 2.6). A two-level-atom Lambda iteration,
 * S_L = (1 - eps) Jbar + eps B (Sect. 2.1, Eq. 3), runs on top.
 *
 * Conventions shared by every entry point:
 *   - Status codes: every function returns vrt_status (0 = success, 1 = a
 *     warning with valid outputs, negative = error). No C++ exception crosses
 *     the ABI. After an error, vrt_ctx_last_error() returns a message that
 *     stays valid until the next call on the same context.
 *   - Host vs device pointers: arguments documented "host" are read or written
 *     by the CPU before the call returns. Arguments documented "device" are
 *     HIP device allocations (for instance torch tensors on the context's
 *     GPU); the library only enqueues work on the context's stream, so the
 *     caller must keep them alive until that stream has completed.
 *   - Layout: per-(site, wavelength) arrays are C-contiguous [site][lambda]
 *     with lambda fastest, in the caller's site order. Per-ray intensities are
 *     [ray][site][lambda]. Sizes are int64, indices int32 (n < 2^31).
 *   - Precision: VRT_F64 arrays are double, VRT_F32 arrays are float.
 *   - Ownership: the caller owns every buffer it passes; host geometry is
 *     copied when a grid is created. A context owns its grids' schedules,
 *     scratch memory and captured HIP graphs; destroying a grid or the
 *     context frees them. One context must not be used from two host threads
 *     at once; separate contexts are independent.
 */
#ifndef VRT_H
#define VRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vrt_status;

#define VRT_OK 0
#define VRT_W_NOT_CONVERGED 1 /* iteration cap reached; outputs valid */
#define VRT_E_ARG (-1)        /* null pointer, bad size or bad enum */
#define VRT_E_GRID (-2)       /* malformed neighbour lists, walls or geometry */
#define VRT_E_DAG (-3)        /* the upwind graph of a ray is not acyclic */
#define VRT_E_HIP (-4)        /* a HIP runtime call failed */
#define VRT_E_NOMEM (-5)      /* device or host allocation failed */
#define VRT_E_NUMERIC (-6)    /* NaN, Inf or negative opacity; NaN source change */
#define VRT_E_STATE (-7)      /* call out of order (e.g. no rays set yet) */
#define VRT_E_TIMEOUT (-8)    /* a bounded device-side wait gave up; outputs invalid */

typedef enum { VRT_F64 = 0, VRT_F32 = 1 } vrt_prec;

/* How a formal solution is launched.
 * PLAIN:      one kernel per (ray, level) of the upwind schedule, rays in turn.
 * BATCHED:    one kernel per level step with all rays in flight together.
 * GRAPH:      BATCHED, captured once into a HIP graph and replayed.
 * PERSISTENT: one kernel for all rays and levels (Voronoi grids; regular
 *             grids fall back to GRAPH). Into caller rows (I_rays) each site
 *             waits for the completion stamps of its upwind sites. Into the
 *             library's own rows (I_rays NULL, linear segment) readiness rides
 *             in the sign bit: odd epochs store -I, and a site waits until the
 *             upwind elements it loads carry its epoch's sign; the J quadrature
 *             and vrt_emergent_gather read those rows as |I|. That encoding
 *             needs I >= 0 (S, I_bottom, I_top >= 0); a negative or NaN
 *             intensity is reported as VRT_E_NUMERIC. Rows pass between
 *             wavefronts through buffer descriptors; when one ray's rows
 *             reach 4 GiB, each access uses the descriptor of its 2 GiB window
 *             (same results, a few more instructions per access). Check vrt_grid_device_status
 *             after synchronising to learn whether a bounded wait gave up
 *             (VRT_E_TIMEOUT) or a value could not be encoded (VRT_E_NUMERIC).
 * AUTO:       the mode vrt_grid_autotune chose for the grid (GRAPH until the
 *             autotuner has run on it). */
typedef enum {
  VRT_EXEC_PLAIN = 0,
  VRT_EXEC_BATCHED = 1,
  VRT_EXEC_GRAPH = 2,
  VRT_EXEC_PERSISTENT = 3,
  VRT_EXEC_AUTO = 4
} vrt_exec;

typedef struct vrt_ctx_s *vrt_ctx;
typedef struct vrt_grid_s *vrt_grid;

/* Library version string (static storage). */
const char *vrt_version(void);

/* Human-readable name of a status code (static storage). */
const char *vrt_status_string(vrt_status s);

/* Host-only check of Voronoi grid geometry (Sect. 2.4: cells, neighbours,
 * Delaunay lines). Checks that nbr_ptr is non-decreasing from 0 to m, that
 * every neighbour index is in [0, n), that shifts are in {-1, 0, 1} (and 0 when
 * not periodic), that no site is its own neighbour with a zero shift, that the
 * lists are symmetric (i -> (k, s) implies k -> (i, -s)), that wall flags use
 * only bits 0 and 1, and that sites lie inside [lo, hi]. Runs no GPU code.
 * msg (host, may be NULL) receives up to msg_len bytes describing the first
 * problem found. Returns VRT_OK or VRT_E_GRID / VRT_E_ARG. */
vrt_status vrt_validate_voronoi(int64_t n, const double *xyz, const int64_t *nbr_ptr,
                                const int32_t *nbr_idx, const int8_t *nbr_shift,
                                const uint8_t *wall, const double lo[3], const double hi[3],
                                uint32_t periodic_xy, char *msg, int64_t msg_len);

/* Create a context on HIP device `device`, enqueuing on `stream` (a
 * hipStream_t; NULL = the device's null stream). */
vrt_status vrt_ctx_create(int32_t device, void *stream, vrt_ctx *out);
/* Destroys the context and every grid still alive on it (their handles
 * become invalid). */
void vrt_ctx_destroy(vrt_ctx ctx);
const char *vrt_ctx_last_error(vrt_ctx ctx);
/* Switch the stream later calls enqueue on (drops captured graphs). */
vrt_status vrt_ctx_set_stream(vrt_ctx ctx, void *stream);
/* Block until all work the context has enqueued has finished. */
vrt_status vrt_ctx_synchronize(vrt_ctx ctx);

/* Kernel timing. While profiling is on, formal solutions launched with
 * VRT_EXEC_PLAIN or VRT_EXEC_BATCHED record a pair of HIP events on the
 * context stream around every kernel (graph replays are not instrumented).
 * vrt_ctx_profile() waits for the recorded events and returns the totals of
 * one kernel class since the last reset:
 *   kernel 0 = Voronoi sweep, 1 = angle quadrature of J, 2 = regular-grid sweep;
 *   ms = summed kernel time, launches = number of launches, units = summed
 *   site * ray * wavelength updates (for kernel 1: site * wavelength outputs
 *   times rays). Any output pointer may be NULL (host). */
vrt_status vrt_ctx_set_profiling(vrt_ctx ctx, int32_t on);
vrt_status vrt_ctx_profile(vrt_ctx ctx, int32_t kernel, double *ms, int64_t *launches, int64_t *units);
vrt_status vrt_ctx_profile_reset(vrt_ctx ctx);

/* Voronoi grid (Sect. 2.4, 2.5). All pointers host; copied.
 *   xyz       [n][3] site positions (m).
 *   nbr_ptr   [n+1], nbr_idx [m]: CSR neighbour lists (Voronoi cells sharing a face).
 *   nbr_shift [m][2] periodic image of the neighbour, in {-1,0,1}: the image of
 *             site k adjacent to i sits at r_k + (sx*Lx, sy*Ly, 0). May be NULL
 *             when periodic_xy is 0.
 *   wall      [n]: bit 0 = the cell touches the bottom wall z = lo[2], bit 1 =
 *             the top wall z = hi[2]. Sites whose cell touches the upwind wall
 *             of a ray are that ray's boundary sites (rays start at the bottom
 *             or top boundary, Sect. 2.5).
 *   lo, hi    box corners; the periods are Lx = hi[0]-lo[0], Ly = hi[1]-lo[1].
 * Runs vrt_validate_voronoi first and returns its status on failure. */
vrt_status vrt_grid_create_voronoi(vrt_ctx ctx, int64_t n, const double *xyz,
                                   const int64_t *nbr_ptr, const int32_t *nbr_idx,
                                   const int8_t *nbr_shift, const uint8_t *wall,
                                   const double lo[3], const double hi[3], uint32_t periodic_xy,
                                   vrt_grid *out);

/* Regular grid for short characteristics (Sect. 2.6). Points (i*dx, j*dy,
 * z[k]), periodic in x and y with periods nx*dx and ny*dy; z (host [nz]) is
 * strictly increasing. Site index = (k*ny + j)*nx + i. */
vrt_status vrt_grid_create_regular(vrt_ctx ctx, int32_t nx, int32_t ny, int32_t nz, double dx,
                                   double dy, const double *z, vrt_grid *out);

/* Drains the context stream and frees the grid. Must not be called after its
 * context was destroyed (that already freed it). */
void vrt_grid_destroy(vrt_grid grid);

/* Set the angle quadrature (Sect. 2.5: a fixed quadrature of directions).
 *   dir [n_rays][3] unit vectors (host), none horizontal; w [n_rays] weights
 *   (host), positive, summing to 1 within 1e-12, so J = sum_r w_r I_r.
 *   r_exp: exponent r of the line weights (Eq. 6); the paper uses 7.
 * On a Voronoi grid this selects, on the GPU, the two upwind Delaunay lines of
 * every (ray, site) (Eq. 5-6), builds each ray's level schedule (a site's
 * level is one more than the largest level of the sites it reads from;
 * boundary sites have level 0), orders sites by (level, index) and packs the
 * per-(ray, site) records in sweep order. Blocks until done. Returns
 * VRT_E_GRID if a non-boundary site has no neighbour upwind in height,
 * VRT_E_DAG if a schedule does not close. */
vrt_status vrt_grid_set_rays(vrt_grid grid, int32_t n_rays, const double *dir, const double *w,
                             double r_exp);

/* Launch and layout knobs of a grid (used by the autotuner; defaults in brackets).
 *   VRT_TUNE_RECORD_ORDER  order of the records inside one (level, ray)
 *                          segment: 0 = site index, 1 = Morton order of the
 *                          sites' horizontal position [1]. Takes effect at the
 *                          next vrt_grid_set_rays.
 *   VRT_TUNE_XCD_CHUNKS    0 = plain block order; k > 0 = hand each of k
 *                          consecutive chunks of a launch's records to one of
 *                          k accelerator dies, so neighbouring records share a
 *                          die's L2 [8].
 * Returns VRT_E_ARG for an unknown knob or value. Drops captured graphs. */
#define VRT_TUNE_RECORD_ORDER 1
#define VRT_TUNE_XCD_CHUNKS 2
/*   VRT_TUNE_RAY_AFFINITY   1 = every ray's records run on one die for the
 *                           whole sweep (rays dealt to the 8 dies in
 *                           serpentine order of their level counts), so a
 *                           level reads the rows its predecessor wrote through
 *                           the same L2; overrides VRT_TUNE_XCD_CHUNKS in
 *                           batched and graph sweeps [0]. */
#define VRT_TUNE_RAY_AFFINITY 5
/*   VRT_TUNE_CHAINS         1..8: split the rays of a batched or graph sweep
 *                           into this many contiguous ranges, each swept on a
 *                           stream of its own (forked from and joined to the
 *                           context stream), so the launch latency of one
 *                           range overlaps the work of the others [1]. */
#define VRT_TUNE_CHAINS 6
/*   VRT_TUNE_LANE_BYTES     16 or 32: bytes of a [site][lambda] row each lane
 *                           moves per access in the level-synchronous sweep
 *                           (32 halves the lanes per record and doubles the
 *                           records per wavefront when the row length and the
 *                           arrays' alignment allow it) [16]. */
#define VRT_TUNE_LANE_BYTES 8
/*   VRT_TUNE_RAY_GROUPS     1..64: sweep the rays of a batched or graph sweep
 *                           in this many consecutive passes over contiguous
 *                           ray ranges (fewer rows in flight per level step,
 *                           more launches) [1]. */
#define VRT_TUNE_RAY_GROUPS 9
/*   VRT_TUNE_INTERLEAVE     1 = batched and graph sweeps (without chains, ray
 *                           groups or ray affinity) read a second copy of the
 *                           records in which each level step is ordered by the
 *                           sites' horizontal Morton code across all rays, so
 *                           a die's chunk of a step is a region of the box
 *                           for every ray; 2 = the same copy ordered by site
 *                           index across rays (for sites numbered along space,
 *                           e.g. a batch of atmospheres, whose Morton codes
 *                           would interleave the atmospheres) [0]. The
                           persistent sweep reads the same copy, so one of
                           its wave items mixes rays. */
#define VRT_TUNE_INTERLEAVE 10
/*   VRT_TUNE_PIPELINE       0 = one group of records per wavefront in the
 *                           level-step sweeps; 2, 4 or 8 = each wavefront
 *                           sweeps that many consecutive groups, with the
 *                           next groups' records and rows loaded while one is
 *                           computed (16-byte lanes and rows of at most one
 *                           lane-vector per lane; other layouts keep the
 *                           classic kernel). Results are the same bits. */
#define VRT_TUNE_PIPELINE 14
/*   VRT_TUNE_REGULAR_TILE   regular grids: 1 = every plane after the first
 *                           runs the LDS-tiled kernel (a workgroup stages the
 *                           chi, S and I of the upwind block of an 8 x 8 tile
 *                           of points once and interpolates all four corners
 *                           from LDS; needs 16-byte rows), 0 = the row kernel
 *                           (every point loads its four upwind corners, which
 *                           neighbouring points share through the caches),
 *                           2 = tiled in double precision, rows in single
 *                           (on a 128 x 128 x 256 grid with 64 wavelengths
 *                           the tiles were 5 % faster in FP64 and 12 % slower
 *                           in FP32); identical results [2]. */
#define VRT_TUNE_REGULAR_TILE 15
/*   VRT_TUNE_SHARED_LEVELS  Voronoi grids: 1 = the rays of one hemisphere and
 *                           one horizontal direction (one azimuth, all
 *                           inclinations) share one level schedule, the
 *                           longest path in the union of their dependency
 *                           graphs (acyclic: every line runs strictly upwind in
 *                           height), so a site's records of those rays sit in
 *                           one level step and share its chi and S rows;
 *                           0 = one schedule per ray [0]. Rebuilds the
 *                           schedules and records at once when the rays are
 *                           set; identical results. vrt_grid_schedule then
 *                           reports the shared levels. */
#define VRT_TUNE_SHARED_LEVELS 16
/*   VRT_TUNE_SEGMENT        source model along a Delaunay line (Voronoi grids):
 *                           0 = linear (Sect. 2.5) [0]; 1 = quadratic Bezier
 *                           (the higher-order solver Sect. 2.5 points to, de
 *                           la Cruz Rodriguez & Piskunov 2013): I = e^-x I_k +
 *                           alpha S_k + beta S_i + gamma C, with the control
 *                           value C = S_i - x S'_i / 2 from the Fritsch-Butland
 *                           mean of the upwind slope and the slope along the
 *                           site's downwind lines (the Eq. 5-6 selection for the
 *                           opposite direction), kept between S_k and S_i.
 *                           Formal solutions and plain (accel = 0) two-level
 *                           iterations in every execution mode; the reverse
 *                           sweep, the accelerated iteration and the autotuner
 *                           return VRT_E_ARG with it. */
#define VRT_TUNE_SEGMENT 11
/*   VRT_TUNE_REVERSE_PERSISTENT 1 = the reverse sweep of vrt_formal_solution_vjp
 *                           runs each ray group as one persistent launch (the
 *                           dataflow of the persistent sweep run backwards:
 *                           a site waits for the stamps of the sites that read
 *                           it in the forward sweep); identical results [0].
 *                           Check vrt_grid_device_status afterwards. */
#define VRT_TUNE_REVERSE_PERSISTENT 13
/*   VRT_TUNE_SPIN_CAP       bound on the polls of one wait in the persistent
 *                           sweep [2^22]; a wait that exceeds it gives up.
 *   VRT_TUNE_PERSIST_BLOCKS workgroups of the persistent sweep, 1 .. 2^20
 *                           [0 = as many as the runtime reports can be
 *                           resident]; any count gives the same results
 *                           (workgroups that are not resident when the
 *                           others start take no work). */
#define VRT_TUNE_SPIN_CAP 3
#define VRT_TUNE_PERSIST_BLOCKS 4
vrt_status vrt_grid_tune(vrt_grid grid, int32_t knob, int64_t value);

/* Autotuner: times candidate launch settings on a formal solution with the
 * given arguments (as for vrt_formal_solution): for each record order, the
 * graph-launched level steps under a fixed list of {die chunks, ray
 * affinity, lane bytes, interleaved record copy (Morton or site order),
 * pipeline depth} settings, and (Voronoi grids, linear segment) the
 * persistent sweep; then, with levels shared by the rays of one azimuth
 * (VRT_TUNE_SHARED_LEVELS), the layouts that pay with them; `reps` replays
 * each after one warm-up. Keeps the fastest
 * setting on the grid, including its launch mode for VRT_EXEC_AUTO, and
 * writes a one-line JSON report (host, may be NULL) of every candidate's mean
 * time in ms and the choice. A candidate that fails (e.g. a device error of
 * the persistent sweep) is reported with "ms": null and skipped. On a regular
 * grid the candidates are the graph-launched plane steps with the row kernel
 * and with the LDS-tiled kernel (VRT_TUNE_REGULAR_TILE 0 and 1).
 * Re-packs the sweep records when the record order changes. When the choice
 * is not the persistent sweep, the library's sign-encoded intensity rows that
 * its candidates used are freed (n_rays x n x n_lambda elements; a later
 * persistent solution allocates them again). Blocks. */
vrt_status vrt_grid_autotune(vrt_grid grid, vrt_prec prec, int32_t n_lambda, const void *chi,
                             const void *S, const void *I_bottom, const void *I_top, void *J,
                             void *I_rays, int32_t reps, char *report, int64_t report_len);

/* Sizes of a grid: number of sites, rays, the largest level count over rays
 * (number of planes on a regular grid) and the number of (ray, site) pairs
 * that fell back to the best z-upwind line because no neighbour lay ahead of
 * the ray. Any output pointer may be NULL (host). */
vrt_status vrt_grid_info(vrt_grid grid, int64_t *n_sites, int32_t *n_rays, int32_t *max_levels,
                         int64_t *n_fallback);

/* Copy one ray's upwind selection and schedule to the host (all [n] unless
 * stated; any pointer may be NULL):
 *   k1, k2   chosen upwind sites (-1 = none; both -1 at boundary sites),
 *   w1       weight of k1 (k2 gets 1 - w1), ds1, ds2 Delaunay line lengths,
 *   level    level of each site, order sites sorted by (level, index),
 *   level_ptr [n_levels + 1] first position of each level in order,
 *   n_levels number of levels. Voronoi grids only. Blocks. */
vrt_status vrt_grid_schedule(vrt_grid grid, int32_t ray, int32_t *k1, int32_t *k2, double *w1,
                             double *ds1, double *ds2, int32_t *level, int32_t *order,
                             int32_t *level_ptr, int32_t *n_levels);

/* Grey LTE continuum (Sect. 2.1 with S = B; opacity recipe of the synthetic
 * atmosphere): chi = kappa0 * rho^2 * T^9 at every wavelength and
 * S = B_lambda(T), the Planck function in kW m^-2 nm^-1 sr^-1.
 *   lambda_m (host [n_lambda]) wavelengths in metres; T, rho (device [n],
 *   double); chi, S (device [n][n_lambda], prec). Enqueued, not blocking. */
vrt_status vrt_lte_continuum(vrt_grid grid, vrt_prec prec, int32_t n_lambda,
                             const double *lambda_m, double kappa0, const double *T,
                             const double *rho, void *chi, void *S);

/* vrt_lte_continuum with rows ld_src apart: the chi and S rows of site i start
 * at chi + i * ld_src and S + i * ld_src (elements; ld_src >= n_lambda, and
 * ld_src = n_lambda is vrt_lte_continuum). With S = chi + n_lambda and
 * ld_src = 2 * n_lambda each site's two rows sit side by side, the layout
 * vrt_formal_solution_ld reads fastest. Entries between the rows are not
 * written. Errors: VRT_E_ARG for ld_src < n_lambda and as vrt_lte_continuum. */
vrt_status vrt_lte_continuum_ld(vrt_grid grid, vrt_prec prec, int32_t n_lambda, int64_t ld_src,
                                const double *lambda_m, double kappa0, const double *T,
                                const double *rho, void *chi, void *S);

/* Formal solution for every ray and wavelength and the mean intensity
 * J = sum_r w_r I_r (Sect. 2.1, Eq. 2 and 4; Sect. 2.5, Eq. 5).
 *   chi, S     device [n][n_lambda] opacity (m^-1, >= 0) and source function.
 *   I_bottom   device [n][n_lambda] intensity entering at the bottom boundary
 *              on upward rays; NULL = S (thermalised boundary).
 *   I_top      device [n][n_lambda] entering at the top on downward rays;
 *              NULL = 0.
 *   J          device [n][n_lambda] output; accumulated in double precision.
 *   I_rays     device [n_rays][n][n_lambda] output of every ray's intensity,
 *              or NULL to keep it in library-owned scratch.
 * All arrays use `prec`. Enqueued on the context stream, not blocking. With
 * VRT_EXEC_GRAPH the launch sequence is captured on first use for each set of
 * pointers and replayed afterwards. */
vrt_status vrt_formal_solution(vrt_grid grid, vrt_prec prec, vrt_exec exec, int32_t n_lambda,
                               const void *chi, const void *S, const void *I_bottom,
                               const void *I_top, void *J, void *I_rays);

/* vrt_formal_solution (Sect. 2.1, Eq. 2 and 4; Sect. 2.5, Eq. 5) with input
 * rows ld_src elements apart: the rows of site i of chi, S, I_bottom and I_top
 * start at i * ld_src (ld_src >= n_lambda; ld_src = n_lambda is
 * vrt_formal_solution). J and I_rays keep rows of n_lambda entries. The
 * intended use pairs a site's opacity and source rows, S = chi + n_lambda and
 * ld_src = 2 * n_lambda (one [n][2][n_lambda] array): a sweep reads chi and S
 * of every upwind site together, and paired rows make that one contiguous
 * span; the two-level iteration stores its rows this way. The results are
 * those of vrt_formal_solution on the same values bit for bit. With I_bottom
 * NULL the bottom boundary reads S at the same stride. Errors: VRT_E_ARG for
 * ld_src < n_lambda, for ld_src != n_lambda on a regular grid (its plane
 * kernels read rows of n_lambda entries), and as vrt_formal_solution. */
vrt_status vrt_formal_solution_ld(vrt_grid grid, vrt_prec prec, vrt_exec exec, int32_t n_lambda,
                                  int64_t ld_src, const void *chi, const void *S,
                                  const void *I_bottom, const void *I_top, void *J, void *I_rays);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * formal solution as vrt_formal_solution in the VRT_EXEC_BATCHED mode (the
 * same kernels, so the same J bit for bit), with the per-ray intensities in a
 * static device buffer of the library (64 MiB per GPU, held until the process
 * ends) instead of memory allocated on first use. Calls no hipMalloc, hipFree
 * or other allocating routine. Arguments as for vrt_formal_solution without
 * exec and I_rays; the grid must have its rays set (the schedules are built
 * there). Every call on one GPU shares that buffer, so calls that overlap on a
 * GPU (other streams, other threads) race. The intensities are not kept for
 * vrt_emergent_gather afterwards (pass I_rays there). Errors:
 *   VRT_E_ARG   sizes beyond the buffer (n_rays x n x n_lambda x element size
 *               above 64 MiB), bad precision or n_lambda, null chi, S or J,
 *               or a Voronoi grid tuned to split launch chains (those create
 *               streams);
 *   VRT_E_STATE rays not set. */
vrt_status vrt_formal_solution_noalloc(vrt_grid grid, vrt_prec prec, int32_t n_lambda, const void *chi,
                                       const void *S, const void *I_bottom, const void *I_top, void *J);

/* Reverse-mode derivative (vector-Jacobian product) of vrt_formal_solution on
 * a Voronoi grid, for gradients of a misfit of the intensities (Sect. 2.1 Eq.
 * 2, Sect. 2.5 Eq. 5 differentiated by hand). Given
 *   dL_dI   device [n_rays][n][n_lambda], dL/dI of every ray (may be NULL),
 *   dL_dJ   device [n][n_lambda], dL/dJ (may be NULL; at least one of the two),
 * and the forward inputs chi, S, I_bottom (NULL = S), I_top (NULL = 0) and
 * I_rays (device [n_rays][n][n_lambda], the forward intensities; NULL = the
 * library recomputes them), writes dL/dchi, dL/dS, dL/dI_bottom and
 * dL/dI_top (device [n][n_lambda] each; any may be NULL). When the forward
 * solution used I_bottom = S, the total sensitivity to S is dL_dS +
 * dL_dIbottom. Upwind selection and weights depend on geometry only, so no
 * derivative flows through them. The reverse sweep walks the level steps
 * downwards with each site gathering from the sites that read it (no atomics);
 * sums over rays are double precision.
 *   ray_group  0 = all rays at once; g > 0 = g rays at a time, recomputing
 *              their forward intensities when I_rays is NULL, so the scratch
 *              memory scales with g instead of n_rays (checkpointing by ray
 *              group, for memory-bound cases).
 *   checkpoint_levels  0 = keep the recomputed forward intensities of every
 *              level step (I_rays NULL: a ray group's full rows); k > 0 =
 *              per-level-chunk checkpoints: the level steps are cut into
 *              chunks of k; a first forward pass keeps only the rows that a
 *              later chunk reads (the frontier), and the reverse sweep
 *              recomputes each chunk's rows from them just before its own
 *              reverse steps, in one buffer the size of the largest chunk.
 *              Forward work about doubles; the rows held drop from
 *              group x n to (largest chunk + frontier), both much smaller for
 *              k well below the level count. The results are bit-identical
 *              to k = 0 with the same ray_group. Ignored when I_rays is given
 *              (nothing is recomputed); the reverse sweep then always runs
 *              as level-step launches. The plan (one int4 per sweep record)
 *              is built on the host on first use for each (k, ray_group).
 * Enqueued, not blocking (building a plan blocks). Errors: VRT_E_ARG for a
 * negative ray_group or checkpoint_levels. */
vrt_status vrt_formal_solution_vjp(vrt_grid grid, vrt_prec prec, int32_t n_lambda, const void *chi,
                                   const void *S, const void *I_bottom, const void *I_top,
                                   const void *I_rays, const void *dL_dI, const void *dL_dJ,
                                   void *dL_dchi, void *dL_dS, void *dL_dIbottom, void *dL_dItop,
                                   int32_t ray_group, int32_t checkpoint_levels);

/* Identifier of the grid's last solution: it changes with every formal
 * solution and two-level solve (and when rays are set or a device error is
 * acknowledged), so a caller that reads it right after a formal solution can
 * later name that solution to vrt_formal_solution_vjp_last. Host, immediate. */
vrt_status vrt_grid_solution_id(vrt_grid grid, int64_t *id);

/* vrt_formal_solution_vjp with the forward intensities of the grid's last
 * formal solution instead of recomputed ones: `solution_id` is the value
 * vrt_grid_solution_id returned right after that solution, which must have
 * kept its rows in the library (I_rays NULL) with n_lambda wavelengths; it may
 * have run in either precision (the rows are converted to prec, the sign-
 * encoded rows of the persistent sweep read as |I|). The caller vouches that
 * chi, S and the boundary intensities are that solution's fields in prec (the
 * reverse sweep of Eq. 2 and 5 is then linearised about those rows). All
 * rays' converted rows take n_rays x n x n_lambda values of scratch besides
 * the reverse sweep's own. If that solution's persistent sweep raised a device
 * error, the outputs are NaN (as J is there). Enqueued, not blocking. Errors:
 * VRT_E_STATE when the last solution is another one (any later solve, rays
 * set or error acknowledged), kept no rows of its own, or had another
 * wavelength count; otherwise as vrt_formal_solution_vjp. */
vrt_status vrt_formal_solution_vjp_last(vrt_grid grid, vrt_prec prec, int32_t n_lambda, const void *chi,
                                        const void *S, const void *I_bottom, const void *I_top,
                                        const void *dL_dI, const void *dL_dJ, void *dL_dchi, void *dL_dS,
                                        void *dL_dIbottom, void *dL_dItop, int32_t ray_group,
                                        int64_t solution_id);

/* Device bytes that vrt_formal_solution_vjp holds as scratch for these
 * settings (keep_intensities != 0: the caller passes I_rays; else the forward
 * intensities are recomputed, with checkpoint_levels as there): the adjoint
 * rows of a ray group, the double accumulators, and the recomputed rows
 * (a ray group's full rows, or the largest level chunk plus the frontier and
 * the checkpoint plan). Builds the checkpoint plan when needed (host, blocks).
 * Lets a caller pick ray_group and checkpoint_levels for a memory budget.
 * Errors: VRT_E_ARG (bad arguments, regular grid), VRT_E_STATE (rays not set). */
vrt_status vrt_formal_solution_vjp_scratch(vrt_grid grid, vrt_prec prec, int32_t n_lambda,
                                           int32_t keep_intensities, int32_t ray_group,
                                           int32_t checkpoint_levels, int64_t *bytes);

/* Adjoint of vrt_emergent_gather: writes dL_dI (device [n_rays][n][n_lambda])
 * with dL_dIem (device, layout of vrt_emergent_gather's output) at the
 * emergent rows and zero elsewhere. Enqueued. */
vrt_status vrt_emergent_scatter(vrt_grid grid, vrt_prec prec, int32_t n_lambda, const void *dL_dIem,
                                void *dL_dI);

/* Adjoint of vrt_lte_continuum (with I_bottom = S = B_lambda(T)):
 *   dL/dT   = sum_lambda dL/dchi 9 chi / T + (dL/dS + dL/dI_bottom) dB/dT,
 *   dL/drho = sum_lambda dL/dchi 2 chi / rho,
 * summed over wavelengths in double precision. dL_dchi, dL_dS, dL_dIbottom
 * (may be NULL) are device [n][n_lambda] in `prec`; T, rho, dL_dT, dL_drho
 * are device [n] double. kappa0 is a constant of the recipe, not
 * differentiated. Enqueued. */
vrt_status vrt_lte_continuum_vjp(vrt_grid grid, vrt_prec prec, int32_t n_lambda,
                                 const double *lambda_m, double kappa0, const double *T,
                                 const double *rho, const void *dL_dchi, const void *dL_dS,
                                 const void *dL_dIbottom, double *dL_dT, double *dL_drho);

/* Two-level-atom Lambda iteration (Sect. 2.1, Eq. 3 and 4; stop rule near
 * 1e-3, Sect. 3.3) with a grey continuum beside the line:
 *   chi_lambda = chi_cont + chi_line phi_lambda,
 *   S_lambda   = (chi_line phi_lambda S_line + chi_cont B) / chi_lambda,
 *   Jbar       = sum_lambda wlam_lambda phi_lambda J_lambda,
 *   S_line    <- (1 - eps) Jbar + eps B,
 * repeated until max_i |dS_line| / |S_line| < tol or max_iter iterations. The
 * bottom boundary of upward rays is thermalised (I = B), the top is empty.
 * The formal solutions run in `sweep_prec` with `exec` (VRT_EXEC_GRAPH
 * captures one iteration and replays it); assembly, Jbar, the update and the
 * convergence test are double precision. The library's scratch holds each
 * site's chi and S rows side by side (rows of n_lambda rounded up to 16 bytes)
 * and the per-ray intensities; if the device cannot hold it beside the
 * sign-encoded rows of earlier persistent formal solutions, those are freed.
 *   wlam      host [n_lambda] quadrature weights of the profile.
 *   phi       device [n][n_lambda] double, profile with sum_l wlam phi = 1.
 *   chi_line, chi_cont, B   device [n] double.
 *   S_line    device [n] double: start value in, final value out.
 *   dS_hist   host [max_iter] or NULL: the change after each iteration.
 *   n_iter    host: iterations done.
 *   accel     0: the plain Lambda iteration above. 1 (Voronoi grids): the
 *             Jacobi-accelerated iteration, which divides each correction by
 *             1 - (1 - eps) Lbar_i with Lbar_i = dJbar_i/dS_line,i =
 *             sum_lambda wlam phi (chi_line phi / chi) Lambda*_ii and
 *             Lambda*_ii = sum_r w_r sum_j w_j Psi_0(x_j) the weight of S_i in
 *             I_i along each ray (Eq. 2, 5); computed once per call in double
 *             precision. Same fixed point, far fewer iterations at small eps
 *             (the cure Sect. 2.2 names for eps < 1e-3).
 * Blocks (one small device-to-host read per iteration). Returns VRT_OK when
 * converged, VRT_W_NOT_CONVERGED at the cap, VRT_E_NUMERIC on a non-finite
 * change. Voronoi and regular grids. */
vrt_status vrt_two_level_solve(vrt_grid grid, vrt_prec sweep_prec, vrt_exec exec, int32_t n_lambda,
                               const double *wlam, const double *phi, const double *chi_line,
                               const double *chi_cont, const double *B, double eps, int32_t max_iter,
                               double tol, int32_t accel, double *S_line, double *dS_hist,
                               int32_t *n_iter);

/* Many independent atmospheres solved as one batch (Sect. 3: the method is
 * applied per snapshot; a batch of uneven snapshots shares every launch).
 * The grid is the disjoint union of the atmospheres, atmosphere a owning
 * sites [atm_ptr[a], atm_ptr[a+1]) (host [n_atm+1], from 0 to n, not
 * decreasing; empty atmospheres allowed). No site may select an upwind
 * neighbour in another atmosphere (checked on the device: VRT_E_GRID).
 * The iteration is that of vrt_two_level_solve applied to each atmosphere on
 * its own: the change max |dS_line| / |S_line| is taken per atmosphere, and an
 * atmosphere that has converged keeps its S_line while the others go on, so
 * its result equals a solve of that atmosphere alone.
 *   dS_hist  host [max_iter][n_atm] or NULL: the change of each atmosphere
 *            after each iteration, -1 once it has stopped.
 *   n_iter   host [n_atm], required: iterations done per atmosphere.
 * Other arguments as vrt_two_level_solve. Voronoi grids when n_atm > 1.
 * Returns VRT_OK when every atmosphere converged, VRT_W_NOT_CONVERGED if any
 * reached the cap, VRT_E_NUMERIC on a non-finite change. Blocks. */
vrt_status vrt_two_level_solve_batched(vrt_grid grid, vrt_prec sweep_prec, vrt_exec exec,
                                       int32_t n_lambda, const double *wlam, const double *phi,
                                       const double *chi_line, const double *chi_cont,
                                       const double *B, double eps, int32_t max_iter, double tol,
                                       int32_t accel, double *S_line, int32_t n_atm,
                                       const int64_t *atm_ptr, double *dS_hist, int32_t *n_iter);

/* Wait for the context stream, then report and clear the grid's device error
 * flag: VRT_OK, or VRT_E_TIMEOUT if a bounded wait of a persistent sweep gave
 * up since the last check (the outputs of that solution are invalid). */
vrt_status vrt_grid_device_status(vrt_grid grid);

/* Emergent intensities (Sect. 2.5: rays leave through the far boundary):
 * for each ray, the sites whose cell touches the downwind z-wall (the top
 * wall for upward rays). offsets (host [n_rays+1]) and sites (host
 * [offsets[n_rays]]) describe the lists; either may be NULL to query sizes
 * (offsets alone). Voronoi and regular grids. Blocks. */
vrt_status vrt_grid_emergent_index(vrt_grid grid, int64_t *offsets, int32_t *sites);

/* Gather the emergent intensities of the last formal solution into out
 * (device [offsets[n_rays]][n_lambda], prec), ray by ray in the order of
 * vrt_grid_emergent_index. I_rays is the array given to that formal solution,
 * or NULL if it used library scratch (the last vrt_formal_solution or
 * two-level solve on this grid; then prec and n_lambda must be those of that
 * solution, else VRT_E_ARG). Enqueued. */
vrt_status vrt_emergent_gather(vrt_grid grid, vrt_prec prec, int32_t n_lambda, const void *I_rays,
                               void *out);

/* Final synthesis on the original regular grid (Sect. 2.5, closing paragraph;
 * Sect. 3.2): quantities converged on the Voronoi grid are carried back to
 * the regular points by inverse-distance interpolation from the two nearest
 * sites, and the emergent intensity at mu = 1 follows from long
 * characteristics up each vertical column.
 *
 * vrt_idw_map: for every point p = (i dx, j dy, z[k]) of `regular` (row
 * (k ny + j) nx + i), the two distinct sites of `voronoi` nearest to p and
 * the weight of the nearer one.
 *   Distance: dx = x_p - x_s and dy = y_p - y_s taken to their minimum image
 *   (|d| <= L/2) on a periodic grid, dz = z_p - z_s, d2 = dx^2 + dy^2 + dz^2
 *   (formed without fused multiply-add); ties go to the smaller site index.
 *   Weights u_k = d_k^-power, w1 = u_1 / (u_1 + u_2) (1 when p is a site;
 *   a one-site grid gives idx = (0, 0), w1 = 1).
 *   idx  device [m][2] int32 output (nearest, second nearest),
 *   w1   device [m] double output,
 *   d2   device [m][2] double output of the squared distances, or NULL;
 *   m = nx ny nz. The search walks the neighbour lists, so they must hold
 *   every face neighbour (as vrt_grid_create_voronoi expects).
 * Both grids must share a context. A periodic Voronoi grid needs the same
 * periods (nx dx = Lx, ny dy = Ly within 1e-9) and a box starting within half
 * a period of x = y = 0; a non-periodic one must contain every point in x and
 * y; the planes must lie inside [lo[2], hi[2]] (VRT_E_ARG otherwise).
 * Returns VRT_E_GRID if a walk does not settle (incomplete neighbour lists).
 * Blocks. */
vrt_status vrt_idw_map(vrt_grid voronoi, vrt_grid regular, double power, int32_t *idx, double *w1,
                       double *d2);

/* dst[p][c] = w1[p] src[idx[p][0]][c] + (1 - w1[p]) src[idx[p][1]][c] for every
 * regular point p and column c < n_cols: src device [n_sites][n_cols] double
 * on the Voronoi sites, dst device [m][n_cols] double; idx and w1 as written
 * by vrt_idw_map. An index outside the Voronoi grid gives NaN. Enqueued. */
vrt_status vrt_idw_apply(vrt_grid voronoi, vrt_grid regular, int32_t n_cols, const int32_t *idx, const double *w1,
                         const double *src, double *dst);

/* Emergent line intensity at mu = 1 on the regular grid from a two-level
 * solution on the Voronoi grid (the paper's final synthesis):
 *   S_line at each regular point = the vrt_idw_apply interpolation of S_line
 *   (device [n_sites] double) with idx, w1 from vrt_idw_map;
 *   chi_lambda = chi_cont + chi_line phi_lambda,
 *   S_lambda   = (chi_line phi_lambda S_line + chi_cont B) / chi_lambda
 *   at each point, with phi device [m][n_lambda] in `prec` and chi_line,
 *   chi_cont, B device [m] double; then along each column (i, j), from the
 *   bottom plane upwards, I_k = e^-x I_(k-1) + Psi_u(x) S_(k-1) + Psi_0(x) S_k,
 *   x = (chi_(k-1) + chi_k)/2 (z_k - z_(k-1)) (Eq. 2 with S linear).
 *   I_bottom  device [ny nx][n_lambda] in `prec`, or NULL = B of the bottom
 *             point (thermalised, as in the Lambda iteration);
 *   I_top     device [ny nx][n_lambda] output in `prec` (row j nx + i).
 * The column integration runs in `prec`; the interpolation in double. Uses a
 * library buffer of 4 m values owned by the regular grid. Enqueued. */
vrt_status vrt_synthesis_vertical(vrt_grid voronoi, vrt_grid regular, vrt_prec prec, int32_t n_lambda,
                                  const int32_t *idx, const double *w1, const double *S_line, const void *phi,
                                  const double *chi_line, const double *chi_cont, const double *B,
                                  const void *I_bottom, void *I_top);

/* Long characteristics at mu = 1 for given chi and S (device [m][n_lambda],
 * `prec`) on a regular grid, as in vrt_synthesis_vertical (the LTE continuum
 * synthesis of Sect. 3.2). I_bottom device [ny nx][n_lambda] or NULL = S of
 * the bottom point; I_top device [ny nx][n_lambda] output. One launch.
 * Enqueued. */
vrt_status vrt_lc_vertical(vrt_grid regular, vrt_prec prec, int32_t n_lambda, const void *chi, const void *S,
                           const void *I_bottom, void *I_top);

#ifdef __cplusplus
}
#endif

#endif /* VRT_H */
