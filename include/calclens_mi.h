/*
 * calclens_mi.h -- C ABI of the MI355X lens-plane solver.
 *
 * The library implements the hot path of Becker (2013), "CALCLENS: weak
 * lensing simulations for large-area sky surveys" (arXiv:1210.3069):
 *   - the plane Poisson equation on the sphere (Sec. 2.1, eq. lenspoisson),
 *     solved by a spherical-harmonic transform on a coarse HEALPix grid and
 *     refined by multigrid on rotated patches around ray bundles (Sec. 3.2);
 *   - the deflection and shear from 4th-order finite differences, with the
 *     Christoffel terms of App. A, at arbitrary points (Sec. 3.2);
 *   - the multiple-plane propagation of ray directions, positions and
 *     lensing Jacobians (Sec. 2.2, eqs. betaprop, posprop, Atraj, with the
 *     parallel transport of App. B) and the radial interpolation of the
 *     Jacobian to galaxies (App. D, eq. gatraj).
 *
 * Conventions used by every call:
 *   - Pointers named *_dev are device pointers (HIP device memory on the
 *     plan's device); pointers named *_host are host pointers.  The caller
 *     allocates and owns every input and output buffer; the plan owns its
 *     workspace, allocated once in clm_plan_create and freed in
 *     clm_plan_destroy.
 *   - Calls are asynchronous on the given stream (0 = the null stream) and
 *     never synchronise, except clm_plan_sync_status, clm_plan_get_timing,
 *     clm_alm2map and a solve under the epsilon rule (which reads one
 *     counter per V-cycle).  The other solve, evaluation, ray and adjoint
 *     calls launch kernels only (no allocation, memset or host wait), so
 *     they may be captured in a HIP graph once each has run eagerly on the
 *     plan (the first call of a kernel may set its LDS attribute).
 *   - kappa is the standard convergence; the solve uses lap psi = 2 kappa
 *     (the paper's kappa^(m) is twice the standard one, Sec. 2.1), so
 *     psi_lm = -2 kappa_lm / (l (l+1)) with psi_00 = 0 (Sec. 3.2).
 *   - Maps are HEALPix RING order unless stated; a_lm are complex128
 *     (re, im interleaved) in HEALPix order index = m (2 lmax + 1 - m)/2 + l.
 *   - Vectors and tensors on the sphere are given in the orthonormal
 *     (theta-hat, phi-hat) basis at the point: axis 1 = theta-hat (south),
 *     axis 2 = phi-hat (east), as in App. A.
 *   - Argument and shape errors return a status synchronously and launch
 *     nothing.  Conditions found on the device (a ray that left its patch,
 *     a non-finite value) are latched in the plan and reported by
 *     clm_plan_sync_status.  No C++ exception crosses this interface.
 *   - A plan is not thread-safe; use one plan per stream.
 */
#ifndef CALCLENS_MI_H
#define CALCLENS_MI_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct clm_plan_s* clm_plan;

typedef enum {
  CLM_OK = 0,
  CLM_EINVAL = 1,           /* bad argument, size or pointer                 */
  CLM_ENOMEM = 2,           /* workspace allocation failed                   */
  CLM_EHIP = 3,             /* a HIP runtime call or kernel launch failed    */
  CLM_ENOTCONV = 4,         /* epsilon rule not met within mg_max_vcycles    */
  CLM_ERAY_LEFT_PATCH = 5,  /* a point fell outside its bundle's patch       */
  CLM_ENONFINITE = 6,       /* a non-finite value was produced               */
  CLM_EUNSUPPORTED = 7      /* valid request this build does not implement   */
} clm_status;

/* Arithmetic forms.  CLM_BF16X3 and CLM_BF16X6 (Legendre transforms only):
 * each float32 operand is split into bf16 terms, hi + lo (BF16X3) or hi +
 * mid + lo (BF16X6), and the products hi*hi + hi*lo + lo*hi (BF16X3) or
 * hi*hi + hi*mid + mid*hi + hi*lo + lo*hi + mid*mid (BF16X6) are accumulated
 * in float32 on the matrix cores. */
typedef enum { CLM_FP64 = 0, CLM_FP32 = 1, CLM_BF16X3 = 2, CLM_BF16X6 = 3 } clm_precision;
typedef enum { CLM_SOLVER_SHT = 0, CLM_SOLVER_SHT_MG = 1 } clm_solver;
typedef enum { CLM_ORDER_RING = 0, CLM_ORDER_NESTED = 1 } clm_order;

/*
 * Plan description.  Sizes follow Sec. 3.1-3.2: rays on a HEALPix grid of
 * resolution nside_fine, bundles of resolution nside_bundle (a ray's bundle
 * is its NESTED index shifted right by 2 log2(nside_fine/nside_bundle)), an
 * SHT on a HEALPix grid of resolution nside_sht up to lmax, and multigrid
 * patches whose side is patch_factor bundle sizes with patch_cells finest
 * cells per side (Delta theta' = Delta phi').
 */
typedef struct {
  int32_t nside_fine;    /* power of two >= 1: ray / output grid               */
  int32_t nside_sht;     /* power of two, <= nside_fine (SHT solver: == fine)  */
  int32_t lmax;          /* 1 .. 2^20; default 2 * nside_sht                   */
  int32_t nside_bundle;  /* power of two, <= nside_fine                        */
  int32_t patch_factor;  /* patch side / bundle side (Sec. 3.2: 4)             */
  int32_t patch_cells;   /* finest cells per side: power of two, 8..4096       */
  int32_t mg_vcycles;    /* fixed number of V-cycles per solve (>= 1); 0: the
                            epsilon rule below decides per patch             */
  int32_t nu_pre;        /* red-black sweeps before restriction, 1..4          */
  int32_t nu_post;       /* red-black sweeps after prolongation, 1..4          */
  int32_t solver;        /* clm_solver                                         */
  int32_t mg_prec;       /* clm_precision of the multigrid correction          */
  int32_t max_planes;    /* solution slots held by the plan, >= 1              */
  int32_t legendre_prec; /* clm_precision of the Legendre transforms: CLM_FP64
                            (per plane, vector FP64), or CLM_FP32 / CLM_BF16X3
                            / CLM_BF16X6 (matrix cores; the planes of one
                            clm_poisson_solve call are batched as GEMM
                            columns, 16 at a time;
                            the lambda_lm recurrence stays FP64)           */
  int32_t mg_max_vcycles; /* epsilon rule: at most this many V-cycles (>= 1) */
  double mg_eps;         /* epsilon rule (Sec. 3.2): a patch stops after the
                            first V-cycle with ||r_h|| / ||tau|| < mg_eps,
                            r_h = f' - L_h du, tau = L_H(R du) - R(L_h du) on
                            the first coarse level, area-weighted RMS norms;
                            default 0.1.  Used only when mg_vcycles == 0;
                            must be >= 0 in any case                      */
  int32_t adjoint;       /* 1: also allocate the workspace of
                            clm_shear_adjoint / clm_poisson_adjoint (FP64,
                            about 4 x 8 bytes per finest cell); SHT+MG
                            with a fixed mg_vcycles > 0 and
                            analysis_iters = 0 only                       */
  int32_t analysis_iters; /* Jacobi refinements of the analysis, 0..16
                            (default 0): a_lm <- a_lm + A(f - S a_lm), S the
                            synthesis and A the quadrature analysis on the
                            nside_sht grid, which drives HEALPix's inexact
                            quadrature toward the band-limited solution;
                            legendre_prec = CLM_FP64 only                 */
  int32_t mfma_ana_waves; /* matrix-core forms: waves per workgroup of the
                            analysis (8 or 16) and of the synthesis (8, 12
                            or 16); 0 (default): chosen at plan creation by
                            timing each shape on a full batch (kept for
                            later plans of the same device, grid, lmax,
                            form and batch); the choice is readable with
                            clm_plan_get_desc                             */
  int32_t mfma_syn_waves;
  int32_t mfma_der_waves; /* pure-SHT plans of a matrix-core form: waves per
                            workgroup of the derivative synthesis of
                            clm_shear_at_pixels (4 or 8); 0 (default):
                            chosen at plan creation like the two above    */
} clm_plan_desc;

/* Fill *d with the defaults for a fine grid: nside_sht = nside_fine / 8
 * (>= 1), lmax = 2 nside_sht, nside_bundle = max(1, nside_fine / 64),
 * patch_factor 4, patch_cells = max(256, 4 nside_fine / nside_bundle),
 * 4 V-cycles of (2, 2) sweeps, SHT+MG solver, FP32 multigrid, 1 slot. */
clm_status clm_plan_desc_default(clm_plan_desc* d, int32_t nside_fine);

/* Create a plan on HIP device `device`: validates *desc, allocates all
 * workspace and builds the geometry tables (ring tables, Legendre starting
 * values, NESTED/RING maps, patch rotations, multigrid coefficients, and
 * per patch-setup tile its ring ranges and reference azimuth).
 * Synchronises the device once.  *out is NULL on failure. */
clm_status clm_plan_create(const clm_plan_desc* desc, int device, clm_plan* out);
clm_status clm_plan_destroy(clm_plan plan);
const char* clm_status_string(clm_status s);
/* Copy the last error text of the plan (NUL-terminated, truncated to len). */
clm_status clm_plan_last_error(clm_plan plan, char* buf_host, size_t len);
/* Synchronise `stream`, return and clear the status latched by kernels.
 * CLM_ENONFINITE is latched when the sum of a convergence map handed to a
 * solve is not finite (a NaN or infinite pixel) and, under the epsilon
 * rule, when a patch's residual or truncation norm is not finite (that
 * patch then stops); the solve still runs to its end and its outputs carry
 * the non-finite values. */
clm_status clm_plan_sync_status(clm_plan plan, hipStream_t stream);
/* Bytes of device workspace held by the plan. */
size_t clm_plan_workspace_bytes(clm_plan plan);
/* Copy the resolved description (defaults applied) to *out_host. */
clm_status clm_plan_get_desc(clm_plan plan, clm_plan_desc* out_host);

/*
 * Per-stage kernel timing.  When enabled, every kernel launch of the plan is
 * bracketed by two HIP events recorded on the launch stream (the events
 * come from a pool owned by the plan; recording allocates only while the
 * pool grows).  clm_plan_get_timing synchronises, adds up the elapsed time
 * and launch count of each stage since the last reset, writes the stage
 * names as a comma-separated list into names_host (truncated to len) and
 * the totals into ms_host / count_host (max_stages entries), sets
 * *nstages_host, and resets the accumulators.
 */
clm_status clm_plan_set_timing(clm_plan plan, int32_t enable);
clm_status clm_plan_get_timing(clm_plan plan, char* names_host, size_t len, double* ms_host,
                               int64_t* count_host, int32_t max_stages, int32_t* nstages_host);
/* Restrict the timing to the stages named in the comma-separated list
 * stages_host (NULL or "" = every stage), so that a timed run carries events
 * around the launches of interest only.  Takes effect for later launches. */
clm_status clm_plan_set_timing_stages(clm_plan plan, const char* stages_host);
/* The per-stage totals (ms) of clm_plan_get_timing without names or counts:
 * ms_per_stage_host[i] for i < nstages, stage i named by
 * clm_plan_stage_name(plan, i) (0 beyond the stages seen); synchronises and
 * resets the accumulators like clm_plan_get_timing. */
clm_status clm_plan_timings(clm_plan plan, double* ms_per_stage_host, int32_t nstages);
/* Name of timing stage i, or NULL; the string is owned by the plan. */
const char* clm_plan_stage_name(clm_plan plan, int32_t i);

/*
 * Epanechnikov deposition of particles onto a HEALPix map (Sec. 3.2): the
 * kernel K(theta; sigma) proportional to 1 - (theta / sigma)^2 inside the
 * particle's smoothing angle sigma (App. E's normalised kernel), sampled
 * at the pixel centres within sigma of the particle and normalised over
 * them, so that every particle deposits exactly its weight (exact mass
 * conservation); a particle whose sigma reaches no pixel centre deposits
 * all of it in the pixel that contains it.  Adds
 * weight_i W_i(p) / Omega_pix (Omega_pix = 4 pi / (12 nside^2)) into map_dev
 * [12 nside^2] float64, RING order, so that the map holds mass per unit
 * area (convergence when the weights are convergence times steradian).
 * theta_dev, phi_dev, weight_dev, sigma_dev: [npart] float64, angles in
 * radians; sigma <= 0 or non-finite deposits into the own pixel, sigma
 * above pi is taken as pi; particles with a non-finite position are
 * skipped.  The cost grows as sigma^2 (pixels per disc): meant for kernels
 * of a few pixels.  Float64 atomic additions: the last bits depend on the
 * order in which particles land.  Independent of any plan; accumulates, so
 * the caller zeroes the map first; asynchronous on `stream`, no
 * allocation.  Errors: CLM_EINVAL (sizes, pointers, nside not a power of
 * two up to 8192).
 */
/* Particles of one lens plane, caller-owned device arrays of n float64:
 * sky position (theta, phi, radians), weight (convergence times steradian)
 * and Epanechnikov smoothing angle sigma (radians). */
typedef struct {
  const double* theta;
  const double* phi;
  const double* weight;
  const double* sigma;
  int64_t n;
} clm_particles;

clm_status clm_deposit_epanechnikov(const double* theta_dev, const double* phi_dev,
                                    const double* weight_dev, const double* sigma_dev,
                                    int64_t npart, int32_t nside, double* map_dev,
                                    hipStream_t stream);

/*
 * The lens-plane solve from particles (Sec. 3.2): the particles are
 * deposited with the Epanechnikov kernel on the fine grid (as
 * clm_deposit_epanechnikov), which feeds the SHT step exactly as a kappa
 * map given to clm_poisson_solve does (its mean removed, degraded to the
 * SHT grid).  In SHT+MG plans the multigrid source is the particles'
 * deposition on each patch's cells instead of the interpolated fine map:
 * the kernel times the cell area over the cell centres within sigma of the
 * patch grid continued past its faces, normalised to the particle's weight,
 * so that a particle's mass splits exactly between a patch and its outside;
 * f = 2 (mass per area - mean).  The solve's results go to `slot` as with
 * clm_poisson_solve.  The fine map is formed in the plan's multigrid
 * workspace (SHT+MG plans; CLM_EUNSUPPORTED when that holds fewer than
 * 8 x 12 nside_fine^2 bytes) or in its derivative workspace (SHT-only
 * plans).  A partial-sky domain limits the patch deposition to its patches.
 * Cost per particle grows as sigma^2 and, on the patches, with the number
 * of patches its disc reaches (patches overlap: about patch_factor^2).
 * Asynchronous on `stream`; no allocation.  Errors: CLM_EINVAL (pointers,
 * slot), CLM_EUNSUPPORTED as above.
 */
clm_status clm_poisson_solve_particles(clm_plan plan, const clm_particles* particles,
                                       int32_t slot, hipStream_t stream);

/*
 * Synthesis of a real field from a_lm (Sec. 3.2, the SHT synthesis):
 *   f(r, j) = sum_l a_l0 lambda_l0(theta_r)
 *             + 2 Re sum_{m>=1} [sum_l a_lm lambda_lm(theta_r)] e^{i m phi_rj}
 * alm_dev: [nalm(lmax)] complex128; map_dev: [12 nside^2] float64 (RING).
 * Independent of any plan; allocates and frees its own temporary workspace
 * (not for use under stream capture).
 */
clm_status clm_alm2map(const double* alm_dev, int32_t lmax, int32_t nside,
                       double* map_dev, hipStream_t stream);

/*
 * clm_alm2map for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, result and layout as clm_alm2map, but nothing is
 * allocated, freed or synchronised: all tables and intermediates live in a
 * 16 MiB file-scope device array, one per GPU, held by the library until the
 * process ends, and rebuilt by every call on `stream`.  Limits: 1 <= lmax
 * <= 512 and nside a power of two <= 256; larger requests return
 * CLM_EUNSUPPORTED and launch nothing (CLM_EINVAL for null pointers, lmax < 1
 * or an nside that is not a power of two).  Calls on one GPU share that
 * array, so calls that overlap in time on one GPU (other streams, other
 * threads) race and must be ordered by the caller.  Asynchronous on
 * `stream`, so it may be captured in a HIP graph.
 */
clm_status clm_alm2map_noalloc(const double* alm_dev, int32_t lmax, int32_t nside,
                               double* map_dev, hipStream_t stream);

/*
 * The plane Poisson solve (Sec. 3.2).  kappa_dev: [nplanes][12 nside_fine^2]
 * standard convergence, RING order, float64 (kappa_is_fp64 = 1) or float32.
 * Plane p of the batch goes to solution slot first_slot + p
 * (first_slot + nplanes <= max_planes).  Steps per plane:
 *   1. kappa' = kappa - mean(kappa); degrade to nside_sht by the mean of the
 *      NESTED children (mass conserving, Sec. 3.2);
 *   2. analysis a_lm = (4 pi / N_pix) sum_r lambda_lm(theta_r) F_m(r), with
 *      F_m(r) the DFT of ring r at order m (HEALPix aliasing kept);
 *   3. psi_lm = -2 a_lm / (l (l+1)), psi_00 = 0;
 *   4. synthesis of psi on the nside_sht grid;
 *   SHT+MG solver only:
 *   5. per bundle b: rotated patch, u0 = psi_SHT interpolated (HEALPix
 *      linear interpolation) at the cell centres, Dirichlet data psi_SHT on
 *      the patch faces, f = 2 (kappa' interpolated at the cell centres),
 *      f' = f - L u0 in float64;
 *   6. mg_vcycles FAS V-cycles on du = u - u0 (zero on the faces) with
 *      red-black Gauss-Seidel, area-weighted restriction and bilinear
 *      prolongation with injection on the outermost ring, levels down to
 *      4 x 4 solved exactly.
 * Results stay in the slot: psi_lm, the psi_SHT map and (SHT+MG) the patch
 * potential u0 + du.
 */
clm_status clm_poisson_solve(clm_plan plan, const void* kappa_dev, int32_t kappa_is_fp64,
                             int32_t first_slot, int32_t nplanes, hipStream_t stream);

/*
 * The plane Poisson solve of several plans at once, for batches of planes
 * of different grids (nside, lmax) in the matrix-core forms: plans[0 ..
 * nplans-1] (1 <= nplans <= 4, one device, one legendre_prec other than
 * CLM_FP64), kappa_dev[i] the [nplanes[i]][12 nside_fine_i^2] convergence
 * of plan i (float64 if kappa_is_fp64[i], else float32; nplanes[i] <=
 * max_planes of plan i, planes to slots 0 ..).  Per round of up to 16
 * planes of every plan, the Legendre analysis of all plans is one
 * persistent launch (workgroups take (plan, m, ring block) items from a
 * counter, largest first) and so is the synthesis, with the waves per
 * workgroup of plans[0]; the ring transforms and the Poisson step run per
 * plane.  Results as clm_poisson_solve (SHT+MG plans then run their
 * multigrid per plane).  Asynchronous on `stream`, launches kernels only,
 * so it may be captured in a HIP graph.
 */
clm_status clm_poisson_solve_multi(const clm_plan* plans, int32_t nplans,
                                   const void* const* kappa_dev,
                                   const int32_t* kappa_is_fp64, const int32_t* nplanes,
                                   hipStream_t stream);

/* Copies out of a solution slot (device destinations):
 *   psi_alm: [nalm(lmax)] complex128; psi_map: [12 nside_sht^2] float64;
 *   patch potential: [npatch][patch_cells][patch_cells] float64 = u0 + du
 *   of patches (bundles, NESTED index) first_patch .. first_patch+npatch-1. */
clm_status clm_get_psi_alm(clm_plan plan, int32_t slot, double* out_dev, hipStream_t stream);
clm_status clm_get_psi_map(clm_plan plan, int32_t slot, double* out_dev, hipStream_t stream);
clm_status clm_get_patch_potential(clm_plan plan, int32_t slot, int64_t first_patch,
                                   int64_t npatch, double* out_dev, hipStream_t stream);

/*
 * Gradient and covariant Hessian of psi (Sec. 3.2 last paragraphs, App. A):
 *   grad = (d_theta psi, d_phi psi / sin theta)
 *   hess = (U_tt, U_pp, U_tp) with U_tt = psi_tt,
 *          U_pp = psi_pp / sin^2 + cot psi_t, U_tp = psi_tp / sin - cos psi_p / sin^2.
 * shear = ((U_tt - U_pp)/2, U_tp), convergence = (U_tt + U_pp)/2.
 * SHT+MG: 4th-order finite differences of u0 + du at the cells (one-sided
 * stencils within one cell of the patch edge), bilinear interpolation of
 * the raw partials to the point, metric terms at the point, rotation to the
 * global basis.  A point is evaluated in the patch of the bundle that
 * contains it.
 *
 * clm_shear_from_potential: points theta_dev/phi_dev [npts] float64 (SHT+MG
 * solver only).  clm_shear_at_pixels: all 12 nside_fine^2 pixel centres in
 * `order` (both solvers; the SHT solver synthesises the derivatives
 * directly from psi_lm, as clm_shear_at_pixels_batch below).  grad_dev: [2][npts], hess_dev: [3][npts], float64
 * if out_fp64 else float32.  Points whose interpolation footprint leaves
 * their patch get NaN and latch CLM_ERAY_LEFT_PATCH.
 */
clm_status clm_shear_from_potential(clm_plan plan, int32_t slot, const double* theta_dev,
                                    const double* phi_dev, int64_t npts, int32_t out_fp64,
                                    void* grad_dev, void* hess_dev, hipStream_t stream);
clm_status clm_shear_at_pixels(clm_plan plan, int32_t slot, int32_t order, int32_t out_fp64,
                               void* grad_dev, void* hess_dev, hipStream_t stream);

/*
 * The pure-SHT solver's derivative fields for several planes (Sec. 3.2,
 * last paragraph): clm_shear_at_pixels for slots first_slot ..
 * first_slot + nplanes - 1 of an SHT-only plan, into grad_dev
 * [nplanes][2][npix] and hess_dev [nplanes][3][npix] (npix = 12
 * nside_fine^2, `order` RING or NESTED, float64 if out_fp64 else float32).
 * With a matrix-core legendre_prec the synthesis runs on the matrix cores,
 * up to 8 planes per launch, in the float32 form for every matrix-core
 * plan: per (ring, l) the FP64 recurrence generates lambda, d lambda / d
 * theta and the two spin-2 functions (the gamma_1 and gamma_2 parts of the
 * covariant Hessian), rounded to float32; then five ring inverses per
 * plane.  An FP64 plan runs the FP64 synthesis plane by plane.  Errors:
 * CLM_EINVAL for a bad slot range, order or pointer; CLM_EUNSUPPORTED on an
 * SHT+MG plan.  Asynchronous on `stream`; no allocation.
 */
clm_status clm_shear_at_pixels_batch(clm_plan plan, int32_t first_slot, int32_t nplanes,
                                     int32_t order, int32_t out_fp64, void* grad_dev,
                                     void* hess_dev, hipStream_t stream);

/*
 * Ray state (Sec. 2.2), one ray per HEALPix pixel of nside_fine in NESTED
 * order (Sec. 3.1), caller-owned device arrays of n = 12 nside_fine^2:
 *   theta, phi: angular position on the current plane (float64);
 *   beta: [3][n] propagation direction (float64, Cartesian);
 *   A, A_prev: [4][n] lensing Jacobian on the current and previous plane,
 *   row-major 2 x 2 (A11, A12, A21, A22), float32, in the basis at the
 *   ray's current position.
 */
typedef struct {
  double* theta;
  double* phi;
  double* beta;
  float* A;
  float* A_prev;
  int64_t n;
} clm_rays;

/* Galaxies for the radial interpolation of App. D: sky position, comoving
 * distance chi (same units as the plane distances), output A [4][n]
 * float32 written when the galaxy's shell is passed. */
typedef struct {
  const double* theta;
  const double* phi;
  const double* chi;
  float* A;
  int64_t n;
} clm_galaxies;

/* Rays at the pixel centres, beta = n, A = A_prev = I (eqs. betaprop,
 * posprop, Atraj initial conditions). */
clm_status clm_rays_init(clm_plan plan, const clm_rays* rays, hipStream_t stream);

/*
 * Propagate rays through lens planes first_plane .. first_plane+nplanes-1
 * (both solvers).  kappa_dev: [nplanes][12 nside_fine^2] (RING) of those
 * planes.  chi_host: [nchi] comoving distances of all planes of the run,
 * chi_0 .. chi_{N-1}, followed by the final target chi_N (nchi = N + 1);
 * curvature_K in the inverse square of the same unit.  For each plane m the
 * call solves the plane, then for every ray:
 *   g, U at n^(m): SHT+MG, from the ray's bundle patch (slot 0 holds the
 *   plane); pure SHT, the HEALPix four-point interpolation of the gradient
 *   and covariant Hessian at the pixel centres (clm_shear_at_pixels_batch's
 *   fields), each transported from its pixel centre to the ray (App. B).
 *   A pure-SHT plan solves up to 8 planes at once into slots 0 .. 7 (one
 *   matrix-core derivative synthesis; FP64 plans: one plane in slot 0) and
 *   keeps psi_lm only (no psi maps);
 *   d = -(g_t theta-hat + g_p phi-hat);
 *   beta <- R(n x d/|d|, |d|) beta (eq. betaprop, read so that rays bend
 *   toward mass, as eq. disclighttraj requires);
 *   x <- x + lambda beta with |x + lambda beta| = chi_{m+1} (eq. posprop);
 *   A^(m+1) = (1 - c_m) A^(m-1) + c_m A^(m) - d_m U A^(m) (eq. Atraj,
 *   chi_{-1} = 0); A^(m+1) and A^(m) parallel transported to n^(m+1) (App. B).
 * Galaxies (may be NULL) whose shell k (chi between the midpoints around
 * chi_k) satisfies first_plane < k <= first_plane + nplanes get
 * A_g = (1 - w) A^(k-1) + w A^(k), w = D_k D_{k-1,g} / (D_g D_{k-1,k}) (eq.
 * gatraj), with the ray Jacobians taken by HEALPix linear interpolation on
 * the image-plane grid; shell-0 galaxies get A_g = I when first_plane = 0.
 */
clm_status clm_raytrace_planes(clm_plan plan, const void* kappa_dev, int32_t kappa_is_fp64,
                               const double* chi_host, int32_t nchi, int32_t first_plane,
                               int32_t nplanes, double curvature_K, const clm_rays* rays,
                               const clm_galaxies* galaxies, hipStream_t stream);

/*
 * One ray update through an already solved slot (the per-plane step of
 * clm_raytrace_planes without the solve and without galaxies): plane index
 * m, distances chi_host as above.  A pure-SHT plan first synthesises the
 * slot's derivative fields at the pixel centres (one plane).
 */
clm_status clm_ray_update(clm_plan plan, int32_t slot, const double* chi_host, int32_t nchi,
                          int32_t m, double curvature_K, const clm_rays* rays,
                          hipStream_t stream);

/*
 * The reduced galaxy step of App. D (eq. gatraj) for shell k alone, with the
 * rays' current Jacobians taken as A^(k) (rays->A) and A^(k-1)
 * (rays->A_prev): the step clm_raytrace_planes takes after the ray update
 * through plane k - 1 (k = 0: A_g = I).  For callers that drive
 * clm_poisson_solve and clm_ray_update themselves.  Galaxies whose chi lies
 * in shell k (between the midpoints around chi_k; the last shell is open
 * above) get A_g; the others are left untouched.  chi_host, nchi and
 * curvature_K as for clm_raytrace_planes; 0 <= k < nchi.  Asynchronous on
 * `stream`.
 */
clm_status clm_galaxies_shell(clm_plan plan, const double* chi_host, int32_t nchi, int32_t k,
                              double curvature_K, const clm_rays* rays,
                              const clm_galaxies* galaxies, hipStream_t stream);

/*
 * Galaxy images by the grid search (Sec. 2.3, Sec. 3.3, App. D) for the
 * galaxies of shell k (chi between the midpoints around chi_k; the last
 * shell open above), after the ray update through plane k - 1 (rays at
 * chi_k with A^(k) in rays->A and A^(k-1) in rays->A_prev).  The image
 * plane is covered by triangles of ray pixel centres (those of consecutive
 * rings merged in azimuth; two per polar cap).  Each ray is moved from chi_k
 * to the galaxy's chi along its direction (no further deflection, the root
 * of eq. posprop of least |lambda|); a triangle whose three rays there
 * enclose the galaxy (barycentric coordinates >= 0 in the plane tangent at
 * the galaxy, gnomonic projection) gives the image: the same coordinates
 * applied to the triangle's pixel centres.  The search covers the triangles
 * within search_radius (rad, at most 0.02; 0: two fine-pixel sizes) of the
 * predicted image (the galaxy moved by the image - source offset of its
 * pixel's ray), nearest first, then within twice that of the galaxy.  The Jacobian at the image is the
 * HEALPix four-point interpolation of the rays' A^(k-1) and A^(k), each
 * parallel transported to the image (App. B), combined by eq. gatraj, in
 * the (theta-hat, phi-hat) basis at the image.  Shell 0: image = galaxy,
 * A = I.  Outputs for the shell's galaxies: theta_img_dev, phi_img_dev
 * [ngal] float64, found_dev [ngal] int32 (0: no image within the search,
 * NaN outputs) and galaxies->A [4][ngal] float32; other galaxies are left
 * untouched.  chi_host, nchi and curvature_K as for clm_raytrace_planes.
 * Asynchronous on `stream`.
 */
clm_status clm_galaxy_images(clm_plan plan, const double* chi_host, int32_t nchi, int32_t k,
                             double curvature_K, const clm_rays* rays,
                             const clm_galaxies* galaxies, double search_radius,
                             double* theta_img_dev, double* phi_img_dev, int32_t* found_dev,
                             hipStream_t stream);

/*
 * The reduced galaxy step of App. D (eq. gatraj) for the shell the rays
 * have just reached: after a clm_ray_update or clm_raytrace_planes through
 * plane m, the rays hold A^(k) (rays->A) and A^(k-1) (rays->A_prev) for
 * k = m + 1, and the galaxies (theta_dev, phi_dev, chi_dev: [ngal] float64)
 * whose chi lies in shell k get A_g_dev [4][ngal] (float32, row-major 2 x 2);
 * the others are left untouched.  The distances and curvature are those of
 * that latest ray update (kept by the plan).  CLM_EINVAL before the first
 * ray update after plan creation or clm_rays_init.  Asynchronous on
 * `stream`.
 */
clm_status clm_galaxies_reduced(clm_plan plan, const clm_rays* rays, const double* theta_dev,
                                const double* phi_dev, const double* chi_dev, int64_t ngal,
                                float* A_g_dev, hipStream_t stream);

/*
 * Partial sky (Sec. 3.4): run the SHT step over the whole sky but the
 * multigrid step, the shear evaluation and the ray update only over a
 * domain of bundles, so that matter outside the domain still acts on it
 * through the SHT boundary values.  bundles_host: [nbundles] NESTED bundle
 * indices at nside_bundle (any order, duplicates allowed); nbundles = 0
 * restores the whole sky.  After the call, until the next one:
 *   - clm_poisson_solve / clm_raytrace_planes set up and solve the patches
 *     of the domain only; every patch still stops on its own under the
 *     epsilon rule, and clm_get_mg_convergence reports 0 cycles and NaN for
 *     patches outside the domain;
 *   - clm_shear_at_pixels writes the pixels of the domain's bundles and
 *     leaves the others untouched; clm_shear_from_potential gives NaN at
 *     points outside the domain and latches CLM_ERAY_LEFT_PATCH;
 *   - clm_ray_update / clm_raytrace_planes move the rays of the domain's
 *     bundles and leave the others untouched; galaxies are served from the
 *     rays around them, so they belong inside the domain, at least one
 *     bundle from its edge;
 *   - clm_get_patch_potential of a patch outside the domain returns that
 *     patch's last solve;
 *   - the adjoints return CLM_EUNSUPPORTED.
 * SHT+MG plans only (CLM_EUNSUPPORTED otherwise); CLM_EINVAL for an index
 * outside 0 .. 12 nside_bundle^2 - 1.  Synchronises the device (the domain
 * tables are copied from the host); no allocation.
 */
clm_status clm_plan_set_domain(clm_plan plan, const int32_t* bundles_host, int64_t nbundles);

/*
 * Full-sky power spectra of a ray state (Sec. 5): the convergence, the E-
 * and B-modes of the shear and the rotation of eq. invmagmat,
 *   kappa = 1 - (A11 + A22)/2, gamma_1 = (A22 - A11)/2,
 *   gamma_2 = -(A12 + A21)/2, omega = (A12 - A21)/2,
 * as maps on the ray grid: ray p (NESTED pixel p) gives the value at its
 * pixel centre, its Jacobian rays->A transported there first from the
 * ray's position rays->theta/phi (App. B).  kappa and omega are analysed
 * as scalars; the shear by the spin-2 functions of the covariant Hessian
 * (X = (m^2/s^2 - l(l+1)/2) lambda - (z/s) d lambda/d theta,
 * Y = (m/s)(d lambda/d theta - (z/s) lambda)), normalised so that the
 * shear of a potential psi (half the trace-free part of its covariant
 * Hessian) has E_lm = N_l psi_lm / 2, N_l^2 = (l-1) l (l+1) (l+2), and
 * B = 0; E and B are 0 for l < 2.  All in FP64 with the HEALPix quadrature
 * weight 4 pi / N_pix.
 * plan: an SHT-only plan (any Legendre form) whose grid is the rays' grid
 * (rays->n = 12 nside_sht^2, nside_sht <= 2048); lmax from the plan.
 * alm_dev: [4][n_lm] complex float64 (kappa, E, B, omega), HEALPix order;
 * cl_dev: [4][lmax+1] float64, C_l = (|a_l0|^2 + 2 sum_{m>0} |a_lm|^2)/(2l+1).
 * Both caller-owned.  Errors: CLM_EINVAL (pointers, ray count),
 * CLM_EUNSUPPORTED (SHT+MG plan, or nside_sht above 2048).  Uses the
 * plan's derivative workspace; asynchronous on `stream`.
 */
clm_status clm_jacobian_spectra(clm_plan plan, const clm_rays* rays, double* alm_dev,
                                double* cl_dev, hipStream_t stream);

/*
 * Multigrid convergence of the latest SHT+MG solve: per patch (bundle index
 * order) the epsilon ratio after the patch's last V-cycle and the number of
 * V-cycles it ran (device buffers of nbundle FP64 / int32 values).  The
 * ratio is NaN when it was not measured (fixed count, mg_vcycles > 0).  After
 * a clm_poisson_solve of several planes the values are the last plane's.  Under
 * the epsilon rule a patch still above mg_eps after mg_max_vcycles latches
 * CLM_ENOTCONV (returned by clm_plan_sync_status).
 */
clm_status clm_get_mg_convergence(clm_plan plan, double* eps_dev, int32_t* cycles_dev,
                                  hipStream_t stream);

/*
 * Adjoint of the solve (plans created with desc.adjoint = 1, SHT+MG solver).
 * With the geometry and the fixed number of V-cycles the map kappa ->
 * (gradient, covariant Hessian of psi at points) of Sec. 3.2 is linear, so
 * the gradient of any loss of those outputs is its transpose applied to the
 * loss's partial derivatives; no state of the forward solve is used.
 *
 * clm_shear_adjoint accumulates, for npts points (theta, phi: device FP64,
 * same convention as clm_shear_from_potential), dgrad [2][npts] and dhess
 * [3][npts] (U_tt, U_pp, U_tp; device FP64) into the plan's accumulator;
 * it may be called several times.  A point outside its bundle's patch is
 * skipped and latches CLM_ERAY_LEFT_PATCH.  Asynchronous on `stream`.
 *
 * clm_poisson_adjoint writes dkappa [12 nside_fine^2] (device FP64, RING):
 * the transpose of the whole chain (patch setup, V-cycles, evaluation, SHT,
 * degrade, demean) applied to the accumulated values, then clears the
 * accumulator.  `slot` selects the plane whose solve the gradient belongs to
 * (the transpose is the same for every slot).  CLM_EUNSUPPORTED for plans
 * without the adjoint workspace.
 */
clm_status clm_shear_adjoint(clm_plan plan, int32_t slot, const double* theta_dev,
                             const double* phi_dev, int64_t npts, const double* dgrad_dev,
                             const double* dhess_dev, hipStream_t stream);
clm_status clm_poisson_adjoint(clm_plan plan, int32_t slot, double* dkappa_dev,
                               hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* CALCLENS_MI_H */
