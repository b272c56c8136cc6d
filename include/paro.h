/*
 * paro.h -- C ABI of libparo, the MI355X (gfx950) hot path of the parallel
 * orbital-updating (ParO) plane-wave eigensolver.
 *
 * Paper: Y. Pan, X. Dai, S. de Gironcoli, X.-G. Gong, G.-M. Rignanese,
 * A. Zhou, "A parallel orbital-updating based plane-wave basis method for
 * electronic structure calculations", arXiv 1702.04045.
 *
 * The library solves the fixed-potential, Gamma-point, norm-conserving
 * (S = I) discrete eigenproblem H Psi = eps Psi of Section 2.3, eq. (e5),
 * with H = kinetic (1/2)|G|^2 + local potential + Kleinman-Bylander (KB)
 * nonlocal part, on the plane-wave basis of eq. (e2) cut off by eq. (e3).
 * The solver is Algorithm 1 of Section 3 (and Algorithm 2 of Section 4)
 * with the cutoff held fixed, as in all runs of Section 5.
 *
 * Conventions (all entry points)
 *  - Every function returns int32_t: PARO_OK (0) or a negative PARO_E* code.
 *    No exception crosses the ABI.  paro_last_error() returns a message for
 *    the last failure on the calling thread.
 *  - Complex numbers are interleaved (re, im) IEEE doubles, the layout of
 *    C99 double complex and of torch.complex128.
 *  - Orbital blocks are band-major: coefficient g of band b is element
 *    [b * ld + g], ld >= n_g.  The G order is the plan's Miller list order.
 *  - Small dense matrices are column-major.
 *  - "dev" pointers are device memory (hipMalloc'd, e.g. owned by torch);
 *    "host" pointers are host memory.  The library allocates no device
 *    memory: the caller passes the plan buffer and a workspace whose sizes
 *    it queries first, and owns them.  The library keeps no caller pointer
 *    beyond a call except the plan buffer, which must live until
 *    paro_plan_destroy.
 *  - All device work is enqueued on the plan's stream and is asynchronous
 *    to the host, except where stated.  A plan is not thread-safe.
 *  - Numerical failures inside enqueued work cannot be returned
 *    synchronously; they set sticky bits in the plan's device status word,
 *    read with paro_get_status().
 */
#ifndef PARO_H
#define PARO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PARO_ABI_VERSION 1

/* return codes */
#define PARO_OK 0
#define PARO_EINVAL (-1)   /* bad argument: NULL, size <= 0, ld < n_g, non-finite input,
                              Miller list not the cutoff sphere in canonical order */
#define PARO_EALIAS (-2)   /* FFT grid smaller than 4 * n_max + 1 along some axis */
#define PARO_ESIZE (-3)    /* plan buffer or workspace smaller than queried */
#define PARO_EHIP (-4)     /* HIP runtime error (text in paro_last_error) */
#define PARO_EUNSUP (-5)   /* valid input outside what this build supports
                              (FFT length not in the supported set, subspace
                              above the dense eigensolver's 1024, density on a
                              grid above 96 points) */

/* sticky device status bits (paro_get_status) */
#define PARO_F_NEGCURV 1   /* PCG met p^H (H - sigma) p <= 0: sigma not below the spectrum */
#define PARO_F_CHOL 2      /* Rayleigh-Ritz overlap matrix not positive definite */
#define PARO_F_NAN 4       /* a NaN reached a PCG scalar */
#define PARO_F_SYNC 8      /* a dense kernel spread over several work-groups waited longer than its
                              limit for another work-group and stopped: its results are invalid */

/* shift modes of paro_iterate */
#define PARO_SHIFT_FIXED 0     /* sigma = sigma_lb every outer iteration */
#define PARO_SHIFT_ADAPTIVE 1  /* sigma = max(sigma_lb, eps_1 - 0.05 - |r_1|) once |r_1| < 0.1 */

/* arithmetic of the source problems in paro_iterate */
#define PARO_PREC_FP64 0   /* everything in FP64 */
#define PARO_PREC_MIXED 1  /* source problems in FP32 (correction form, see
                              paro_source_solve_mixed); H U, Rayleigh-Ritz,
                              residuals and shifts in FP64 */
#define PARO_PREC_MIXED_BF16 2  /* as PARO_PREC_MIXED, with the projector
                              products of the FP32 applies as split-BF16
                              products (paro_apply_h_f32_bf16) */

/* solver variants of paro_iterate */
#define PARO_VARIANT_PARO 0    /* Algorithm 1: Rayleigh-Ritz on span{u_i} (m = nb) */
#define PARO_VARIANT_MPARO1 1  /* Algorithm 2: Rayleigh-Ritz on span{psi_i, e_i} (m = 2 nb) */
#define PARO_VARIANT_MPARO2 2  /* Algorithm 3: as Algorithm 2 with e_i from the projected
                                  correction equation (I - P_i)(H - sigma_i)(I - P_i) e_i =
                                  (eps_i - H) psi_i, P_i the projector onto psi_i (the shift
                                  sigma_i read for the printed lambda); FP64 only */

typedef void *paro_stream_t; /* a hipStream_t; NULL is the default stream */
typedef struct paro_plan_s *paro_plan;

/* One Kleinman-Bylander projector beta_p (nonlocal part of the
 * pseudopotential, Section 2.2).  Gaussian form in the plane-wave basis:
 *   s   (l = 0):          beta(G) = c exp(-w^2 |G|^2 / 2) exp(-i G.R)
 *   p_a (l = 1, m = a):   beta(G) = c (-i w G_a) exp(-w^2 |G|^2 / 2) exp(-i G.R)
 * a = 0, 1, 2 for x, y, z; c normalises sum_G |beta(G)|^2 = 1 over the
 * sphere.  The nonlocal operator is sum_p d_p beta_p beta_p^H. */
typedef struct {
    double center[3]; /* R, Cartesian bohr */
    int32_t l, m;
    double width;     /* w, bohr, > 0 */
    double d;         /* KB energy d_p, Ha */
} paro_projector;

/* The problem statement (all host memory; copied by paro_plan_create). */
typedef struct {
    double cell[9];          /* lattice vectors a1, a2, a3 as rows, bohr */
    double ecut;             /* plane-wave cutoff, Ha: (1/2)|G|^2 <= ecut, eq. (e3) */
    int32_t grid[3];         /* FFT grid N1, N2, N3 of vloc */
    int64_t n_g;             /* size of the G-sphere */
    const int32_t *miller;   /* host, n_g x 3 Miller indices (n1, n2, n3), G = sum n_d b_d;
                                must be the cutoff sphere in canonical (lexicographic) order,
                                as produced by paro_sphere_enumerate */
    const double *vloc;      /* host, N1*N2*N3 local potential values (Ha), C order
                                [i1][i2][i3], at r = sum_d (i_d / N_d) a_d */
    int32_t n_proj;          /* number of KB projectors, >= 0 */
    const paro_projector *proj; /* host, n_proj entries (may be NULL when n_proj = 0) */
} paro_problem;

typedef struct {
    int64_t n_g;
    int32_t nmax[3];         /* max |n_d| over the sphere */
    int32_t grid[3];
    int32_t n_sticks;        /* (n1, n2) lines transformed along n3: for each n1, every n2
                                between the lowest and highest that hold sphere points */
    int32_t n_proj;
    double omega;            /* cell volume, bohr^3 */
} paro_plan_info;

/* Options of paro_iterate. */
typedef struct {
    int32_t n_outer;         /* outer iterations (Algorithm 1 steps 3-5) to run */
    int32_t n_cg;            /* PCG steps per source problem */
    int32_t n_conv;          /* lowest bands whose convergence counts (<= nb) */
    int32_t shift_mode;      /* PARO_SHIFT_* */
    int32_t variant;         /* PARO_VARIANT_* */
    int32_t initial_rr;      /* 1: first run Rayleigh-Ritz on the trial block (Algorithm 1 step 1) */
    double sigma_lb;         /* lower bound of the spectrum (paro_shift_lower_bound) */
    double tol_res;          /* stop once max_{b < n_conv} |H psi_b - eps_b psi_b| <= tol_res
                                (checked on the device after each outer iteration; 0 = never) */
    int32_t precision;       /* PARO_PREC_FP64, PARO_PREC_MIXED or PARO_PREC_MIXED_BF16 */
} paro_iter_opts;

/* ---------------------------------------------------------------- ABI */

int32_t paro_abi_version(void);
const char *paro_last_error(void);

/* ---------------------------------------------------------------- setup (host) */

/* The cutoff sphere of eq. (e3) at k = 0, in canonical order: lexicographic
 * in (n1, n2, n3).  A point is included iff (1/2)|G|^2 <= ecut (1 + 1e-12).
 * cell: host double[9]; miller: host int32[capacity * 3] or NULL (count
 * only); n_g_out: number of points; nmax_out: host int32[3] or NULL.
 * Returns PARO_ESIZE if capacity < n_g (n_g_out still set). */
int32_t paro_sphere_enumerate(const double *cell, double ecut, int64_t capacity,
                              int32_t *miller, int64_t *n_g_out, int32_t *nmax_out);

/* Smallest FFT grid 2^a * {1, 3, 5} >= 4 nmax_d + 1 along each axis, the
 * size at which the FFT apply of the local potential has no alias on the
 * sphere.  nmax, grid_out: host int32[3]. */
int32_t paro_grid_size(const int32_t *nmax, int32_t *grid_out);

/* Device bytes the plan needs for this problem. */
int32_t paro_plan_bytes(const paro_problem *prob, size_t *bytes);

/* Validate the problem and build the plan in dev_buf (device, >= plan
 * bytes, 256-byte aligned): stick maps, kinetic table, V re-laid for the
 * plane transforms,
 * FFT twiddles and the KB projector matrix B (n_g x n_proj), computed by
 * a device kernel.  Synchronises the stream before returning.
 * Errors: PARO_EINVAL, PARO_EALIAS, PARO_ESIZE, PARO_EUNSUP, PARO_EHIP. */
int32_t paro_plan_create(const paro_problem *prob, void *dev_buf, size_t bytes,
                         paro_stream_t stream, paro_plan *plan_out);
int32_t paro_plan_destroy(paro_plan plan);
int32_t paro_plan_set_stream(paro_plan plan, paro_stream_t stream);
int32_t paro_plan_get_info(paro_plan plan, paro_plan_info *info);

/* Device bytes of the workspace for calls on up to nb bands.
 * Valid for paro_apply_h, paro_source_solve, paro_rayleigh_ritz (m <= 2 nb)
 * and paro_iterate with either variant. */
int32_t paro_workspace_bytes(paro_plan plan, int32_t nb, size_t *bytes);

/* Copy the plan's kinetic table (1/2)|G|^2 (dev double[n_g]) or projector
 * matrix B (dev complex[n_proj][n_g], projector-major) to dev memory;
 * for tests. */
int32_t paro_get_kinetic(paro_plan plan, double *kin_dev);
int32_t paro_get_projectors(paro_plan plan, double *beta_dev);

/* ------------------------------------------------------------ autotuning */

/* Launch choices of the z-plane stage of the local part of H (the n2 / n1
 * transforms and the multiply by vloc, eq. (e5)), per plan and per
 * precision (PARO_PREC_FP64; PARO_PREC_MIXED and PARO_PREC_MIXED_BF16 share
 * the FP32 choice):
 *   schedule  the line schedule of the transforms, 0 <= schedule <
 *             n_schedules: threads per line and radix order.  Grids of 24
 *             to 80 points have 3 (radix orders); 96 points has 3 (0: the
 *             cross-lane lines with two bands' columns in LDS, 1: the same
 *             lines on four lanes each, 2: the same lines with one band's
 *             populated columns in LDS, two work-groups per compute unit);
 *             the others 1.  Another radix order changes the rounding of
 *             the transforms, not what they compute.
 *   bands     bands one work-group takes through its z-plane (1 .. 64).
 *             Results are bitwise the same for every value.
 * A new plan starts at schedule 0 and 4 bands, except FP64 on 96 points:
 * schedule 2 and 2 bands (the fastest measured there).  set_schedule re-lays the
 * plan's potential tables for the new schedule on the plan's stream and
 * waits for it: call it while no work that uses the plan is in flight.
 * Errors: PARO_EINVAL (NULL plan, unknown precision, values out of range). */
int32_t paro_plan_set_schedule(paro_plan plan, int32_t precision, int32_t schedule, int32_t bands);
int32_t paro_plan_get_schedule(paro_plan plan, int32_t precision, int32_t *schedule, int32_t *bands,
                               int32_t *n_schedules);

#define PARO_TUNE_FORCE 1  /* time again even if a plan of this shape was tuned before */

typedef struct {
    int32_t schedule[2];   /* chosen schedule: [0] FP64, [1] FP32 */
    int32_t bands[2];      /* chosen bands per work-group */
    double ms[2];          /* plane-stage time on nb bands with the choice, ms */
    double ms_default[2];  /* the same with a new plan's choice */
    int32_t candidates;    /* configurations timed per precision */
    int32_t cached;        /* 1: both choices came from an earlier tuning of this shape */
} paro_tune_result;

/* Time every (schedule, bands) pair of the plane stage on this plan's own
 * shape with nb bands (in the 64-band chunks the solver uses), for both
 * precisions, and select the fastest (the default unless another is more
 * than 1 % faster).  The choice of a shape (grid, sticks, columns, nb) is
 * kept for the process: a later plan of the same shape takes it without
 * timing unless flags has PARO_TUNE_FORCE.  ws: a workspace of
 * paro_workspace_bytes(nb); its contents are overwritten.  Synchronises the
 * plan's stream; not capturable.  result may be NULL.  Errors: PARO_EINVAL,
 * PARO_ESIZE, PARO_EHIP. */
int32_t paro_plan_autotune(paro_plan plan, int32_t nb, void *ws, size_t ws_bytes, int32_t flags,
                           paro_tune_result *result);

/* ---------------------------------------------------------------- hot path */

/* hpsi_b = (H - shift_b) psi_b for b < nb.  The matrix elements are
 * h_mn = (1/2)|G_m|^2 delta_mn + Vt(n_m - n_n) + sum_p d_p beta_p(G_m)
 * conj(beta_p(G_n)) with Vt the grid DFT of vloc (eq. (e5), read with
 * G_m - G_n), applied through sphere -> stick -> plane FFTs.
 * psi, hpsi: dev complex, band-major, leading dimension ld; may not alias.
 * shift: dev double[nb] or NULL (zero).  ws: dev workspace of at least
 * paro_workspace_bytes(nb) bytes. */
int32_t paro_apply_h(paro_plan plan, int32_t nb, const double *psi, int64_t ld,
                     const double *shift, double *hpsi, void *ws, size_t ws_bytes);

/* H psi in single precision: hpsi_b = (H - shift_b) psi_b with psi, hpsi
 * dev complex64 (interleaved float re, im), band-major, leading dimension
 * ld; FP32 FFTs with an FP32 copy of the potential and FP32 matrix-core
 * projector products (split partial sums added in FP64).  The building
 * block of the mixed-precision source solve; shift and ws as paro_apply_h. */
int32_t paro_apply_h_f32(paro_plan plan, int32_t nb, const float *psi, int64_t ld,
                         const double *shift, float *hpsi, void *ws, size_t ws_bytes);

/* paro_apply_h_f32 with the projector products V_NL psi = B D (B^H psi) of
 * Section 2.2 on the BF16 matrix cores: every FP32 operand x is split into
 * hi = bf16(x) and lo = bf16(x - hi), and a product x y is taken as
 * hi hi + hi lo + lo hi, accumulated in FP32 (the split-K partial sums of
 * B^H psi added in FP64).  Each product is within about 3 x 2^-16 of x y,
 * so the nonlocal part carries a relative error of about 5e-5 (FP32
 * operands: 6e-8); the local part is that of paro_apply_h_f32.  Arguments,
 * layout and errors as paro_apply_h_f32. */
int32_t paro_apply_h_f32_bf16(paro_plan plan, int32_t nb, const float *psi, int64_t ld,
                              const double *shift, float *hpsi, void *ws, size_t ws_bytes);

/* The N independent source problems of Algorithm 1, step 3, read with a
 * shift sigma_b below the spectrum:
 *   (H - sigma_b) u_b = (eps_b - sigma_b) psi_b,
 * each by n_cg steps of Teter-preconditioned CG from u_b = psi_b, with the
 * recurrence residual (r_0 = eps_b psi_b - hpsi_b from the carried H psi).
 * Teter preconditioner K(x) = (27+18x+12x^2+8x^3)/(27+18x+12x^2+8x^3+16x^4),
 * x = (1/2)|G|^2 / tau_b, tau_b = <psi_b|T|psi_b>/<psi_b|psi_b>.
 * A band stops early when p^H (H - sigma) p <= 0 (sets PARO_F_NEGCURV) or
 * when r^H z <= 1e-26 r_0^H z_0.
 * psi, hpsi, u: dev complex band-major (ld); eps, shift: dev double[nb];
 * band_flags: dev int32[nb] or NULL, receives the per-band status bits. */
int32_t paro_source_solve(paro_plan plan, int32_t nb, const double *psi, const double *hpsi,
                          int64_t ld, const double *eps, const double *shift, int32_t n_cg,
                          double *u, int32_t *band_flags, void *ws, size_t ws_bytes);

/* The same source problems with FP32 vectors (the "batched mixed" solve):
 * u_b = psi_b + d_b where d_b, from d_b = 0, takes n_cg Teter-preconditioned
 * CG steps on (H - sigma_b) d_b = eps_b psi_b - hpsi_b, the right-hand side
 * formed in FP64 and stored in FP32, H applied as in paro_apply_h_f32, the
 * CG scalars in FP64.  In exact arithmetic this is the iterate of
 * paro_source_solve (its CG run from u = psi); in floating point the error is
 * about 1e-7 |d_b|.  Arguments, layout and flags as paro_source_solve (FP64
 * psi, hpsi, u). */
int32_t paro_source_solve_mixed(paro_plan plan, int32_t nb, const double *psi, const double *hpsi,
                                int64_t ld, const double *eps, const double *shift, int32_t n_cg,
                                double *u, int32_t *band_flags, void *ws, size_t ws_bytes);

/* Rayleigh-Ritz on span{U} (Algorithm 1, step 4): with W = H U given,
 * S = U^H U, Hs = U^H W, S = L L^H, Hhat = L^-1 Hs L^-H = Y diag(eps) Y^H
 * (ascending), C = L^-H Y; writes the lowest n_keep pairs:
 * eps (dev double[n_keep]), psi = U C, hpsi = W C (dev complex band-major,
 * leading dimension ld, n_keep bands).  U and W: m bands each, ld.
 * Sets PARO_F_CHOL if S is not positive definite (outputs then undefined).
 * m <= 2 * (the nb the workspace was sized for), n_keep <= m. */
int32_t paro_rayleigh_ritz(paro_plan plan, int32_t m, int32_t n_keep, const double *U,
                           const double *W, int64_t ld, double *eps, double *psi, double *hpsi,
                           void *ws, size_t ws_bytes);

/* |hpsi_b - eps_b psi_b| for b < nb into res (dev double[nb]). */
int32_t paro_residual_norms(paro_plan plan, int32_t nb, const double *psi, const double *hpsi,
                            int64_t ld, const double *eps, double *res, void *ws, size_t ws_bytes);

/* Lower bound of the spectrum, written to sigma_dev (dev double[1]):
 * sigma_lb = min_j vloc_j + min(0, lambda_min(V_NL)) - 0.1 (Weyl: kinetic
 * >= 0, the local part is a compression of multiplication by V, and
 * V_NL = B D B^H has the nonzero eigenvalues of L^H D L, B^H B = L L^H).
 * ws sized for at least max(1, ceil(n_proj / 2)) bands. */
int32_t paro_shift_lower_bound(paro_plan plan, double *sigma_dev, void *ws, size_t ws_bytes);

/* ParO at fixed cutoff (Algorithm 1 steps 1, 3, 4, 5; Algorithm 2 for
 * variant MPARO1, Algorithm 3 for MPARO2): up to opts->n_outer outer
 * iterations of nb source problems followed by Rayleigh-Ritz (m = nb, or
 * 2 nb for MPARO1 and MPARO2).  PARO_EUNSUP for MPARO2 in mixed precision.
 * psi: in the trial block (initial_rr = 1) or orthonormal Ritz vectors with
 * hpsi = H psi and eps (initial_rr = 0); out the Ritz vectors.  hpsi, eps:
 * out (in when initial_rr = 0).  sigma: dev double[1], out: the shift the
 * next outer iteration would use.  stats: dev double[(n_outer + 1) *
 * (2 nb + 2)] or NULL; row i (row 0: before the first outer iteration)
 * holds eps (nb), residual norms |H psi_b - eps_b psi_b| (nb), the next
 * shift, and 1.0 when max_{b < n_conv} residual <= tol_res.  When tol_res >
 * 0 the loop stops before an outer iteration once that test passed (one
 * host synchronisation per outer iteration).  In adaptive shift mode a
 * source solve that meets negative curvature is redone with sigma_lb (one
 * host synchronisation per outer iteration).  n_done: host int32 or NULL,
 * the outer iterations run.  ws: paro_workspace_bytes(nb).  nb <= 1024 for
 * ParO and nb <= 512 for MParO I and II (PARO_EUNSUP beyond). */
int32_t paro_iterate(paro_plan plan, int32_t nb, double *psi, double *hpsi, int64_t ld,
                     double *eps, double *sigma, const paro_iter_opts *opts, double *stats,
                     void *ws, size_t ws_bytes, int32_t *n_done);

/* Many independent problems (cells of different grids, sphere sizes and
 * band counts) iterated together: for cell i the same computation as
 * paro_iterate(plans[i], nb[i], psi[i], hpsi[i], ld[i], eps[i], sigma[i],
 * &opts[i], stats ? stats[i] : NULL, ws[i], ws_bytes[i], n_done + i), with
 * bitwise the same results.  Each cell's kernels are enqueued on its plan's
 * stream: plans on different streams run concurrently on the GPU.  Two or
 * more cells of one precision (FP64 or PARO_PREC_MIXED, not MParO II) share
 * grouped launches instead: one launch of each kernel of the source
 * problems (and, for ParO with nb <= 92, of the Rayleigh-Ritz step) covers
 * all cells; these run on the first active cell's stream, ordered against
 * the other cells' streams by events.  Every outer iteration first enqueues
 * the work of all cells and then waits for them once (convergence test,
 * negative-curvature retry) instead of once per cell.  With tol_res = 0 and
 * the fixed shift in every cell and one stream for all plans, the call
 * enqueues kernels only (no event, wait or host memory) and can be
 * captured into a HIP graph.  A cell stops at its own n_outer or tolerance.  Each cell needs
 * its own workspace (paro_workspace_bytes(nb[i]) of its plan); cells that
 * share a plan share its stream and run one after the other.  stats may be
 * NULL, or hold NULL entries; n_done may be NULL.  Errors: as
 * paro_iterate, with the failing cell named in paro_last_error;
 * PARO_EINVAL when two cells share a workspace. */
int32_t paro_iterate_batch(int32_t n_cells, const paro_plan *plans, const int32_t *nb, double *const *psi,
                           double *const *hpsi, const int64_t *ld, double *const *eps, double *const *sigma,
                           const paro_iter_opts *opts, double *const *stats, void *const *ws,
                           const size_t *ws_bytes, int32_t *n_done);

/* Read and clear the sticky status bits (synchronises the plan's stream). */
int32_t paro_get_status(paro_plan plan, int32_t *flags);

/* ---------------------------------------------------------------- profiling */

/* Kernel classes that can be timed with HIP events. */
#define PARO_K_STICK_INV 1   /* sphere -> sticks, inverse transform along n3 */
#define PARO_K_PLANE 2       /* z-plane stage: n2/n1 transforms and the V multiply */
#define PARO_K_STICK_FWD 3   /* sticks -> sphere, forward transform along n3, kinetic term */
#define PARO_K_GEMM_HN 4     /* split-K A^H B partial tiles */
#define PARO_K_GEMM_NN 5     /* A B (+ C) */
#define PARO_K_PCG_UPDATE 6  /* PCG vector update and preconditioner */
#define PARO_K_DENSITY 7     /* z-plane stage of paro_density: n2/n1 transforms and w |psi|^2 */

/* Record a HIP event pair around every launch of one kernel class, on the
 * stream it is launched on, for up to max_launches launches, until
 * paro_profile_stop.  Process-wide (one class at a time); not thread-safe.
 * paro_profile_stop synchronises the recorded events and returns the number
 * of timed launches and their summed duration in milliseconds.  The events
 * are kept per device for the next profile (created on the current device
 * at the start, as many as 2 max_launches).
 * paro_profile_start_sampled times only launches 0, every, 2 every, ... of
 * the class (every >= 1; paro_profile_start is every = 1): each event pair
 * orders the stream around its launch, so sampling keeps that cost off the
 * timed work.  Errors: PARO_EINVAL (bad class, count or stride, a profile
 * already running), PARO_EHIP. */
int32_t paro_profile_start(int32_t kernel, int32_t max_launches);
int32_t paro_profile_start_sampled(int32_t kernel, int32_t max_launches, int32_t every);
int32_t paro_profile_stop(int32_t *launches, double *total_ms);

/* ---------------------------------------------------------------- density */

/* Electron density of a block of orbitals on the FFT grid (Section 2.3,
 * eq. (e2) at the grid points r_j = sum_d (j_d / N_d) a_d, without the
 * 1/sqrt(Omega) normalisation):
 *   rho[j] = sum_b w_b |psi_b(r_j)|^2,  psi_b(r_j) = sum_G c_bG exp(2 pi i n.j / N).
 * For eigenpairs of H this is the Hellmann-Feynman gradient of the
 * weighted band energy with respect to the local potential on the grid:
 *   d (sum_b w_b eps_b) / d vloc[j] = rho[j] / (N1 N2 N3)
 * (the matrix elements of eq. (e5) are (1/N) sum_j vloc[j] exp(-2 pi i
 * (n_m - n_n).j / N)), and the gradient of sum_b w_b <psi_b|V|psi_b> for
 * any block.
 * psi: dev complex band-major, leading dimension ld >= n_g; weights: dev
 * double[nb] or NULL (all 1); rho: dev double[N1 N2 N3], C order
 * [j1][j2][j3] like paro_problem.vloc, overwritten.  Bands are summed in a
 * fixed order: the result is bitwise reproducible.  ws: dev workspace of
 * at least paro_density_workspace_bytes(nb) bytes.  Errors: PARO_EINVAL
 * (NULL, nb <= 0, ld < n_g), PARO_ESIZE (workspace too small). */
int32_t paro_density_workspace_bytes(paro_plan plan, int32_t nb, size_t *bytes);
int32_t paro_density(paro_plan plan, int32_t nb, const double *psi, int64_t ld, const double *weights,
                     double *rho, void *ws, size_t ws_bytes);

/* Derivatives of the nonlocal energy sum_b w_b <psi_b| V_NL |psi_b>,
 * V_NL = sum_p d_p beta_p beta_p^H (Section 2.2, the projectors of
 * paro_projector), with respect to each KB energy d_p and each projector
 * centre R_p; with beta_p(G) proportional to exp(-i G.R_p):
 *   dd[p]      = sum_b w_b |P_pb|^2,  P_pb = beta_p^H psi_b,
 *   dR[3p + a] = sum_b w_b d_p 2 Re(conj(P_pb) Q_pb^a),
 *   Q_pb^a = (-i G_a beta_p)^H psi_b.
 * For eigenpairs these are the Hellmann-Feynman derivatives of the weighted
 * band energy sum_b w_b eps_b; the force on an atom is minus the sum of dR
 * over its projectors, plus the local part (paro_density).
 * psi: dev complex band-major (ld >= n_g); weights: dev double[nb] or NULL
 * (all 1); dd: dev double[n_proj]; dR: dev double[n_proj x 3]; both
 * overwritten (nothing is written when n_proj = 0).  The products run on
 * the FP64 matrix cores with fixed-order split-K sums: the result is
 * bitwise reproducible.  ws: dev, 256-byte aligned, at least
 * paro_projector_gradient_workspace_bytes(nb) bytes.  Errors: PARO_EINVAL
 * (NULL, nb <= 0, ld < n_g, misaligned ws), PARO_ESIZE. */
int32_t paro_projector_gradient_workspace_bytes(paro_plan plan, int32_t nb, size_t *bytes);
int32_t paro_projector_gradient(paro_plan plan, int32_t nb, const double *psi, int64_t ld, const double *weights,
                                double *dd, double *dR, void *ws, size_t ws_bytes);

/* Reverse-mode gradient of the band energy after K truncated outer
 * iterations of Algorithm 1 (Section 3) at a fixed shift:
 *   (eps^0, psi^0) = Rayleigh-Ritz of the trial block (step 1), then K outer
 *   iterations of n_cg PCG steps per source problem and Rayleigh-Ritz
 *   (steps 3 and 4), exactly as paro_iterate with PARO_SHIFT_FIXED and no
 *   tolerance, and E = sum_b w_b eps_b^K.
 * Writes E and its derivatives with respect to the local potential on the
 * grid (dvloc[j] = dE/dvloc[j], C order like paro_problem.vloc) and to the
 * projector centres (dR[3p + a] = dE/dR_p,a), differentiating the truncated
 * map itself (not its converged limit): one checkpoint per outer
 * iteration, each outer iteration recomputed in the backward pass with its
 * PCG iterates kept, then the Rayleigh-Ritz, H U and PCG steps reversed on
 * the device.  The trial block and sigma are constants.
 * trial: dev complex nb bands, leading dimension ld >= n_g; weights: dev
 * double[nb]; energy: dev double[1]; dvloc: dev double[N1 N2 N3]; dR: dev
 * double[3 n_proj] (may be NULL when n_proj = 0); all outputs overwritten.
 * ws: dev, 256-byte aligned, paro_truncated_gradient_workspace_bytes(nb,
 * n_outer, n_cg) bytes (about (n_outer + 4 n_cg + 20) nb n_g 16 bytes).
 * A source problem that stopped early (PCG's stopping rules) is
 * differentiated along that branch: its later steps are the identity.
 * Synchronises the plan's stream.  Errors: PARO_EINVAL, PARO_ESIZE,
 * PARO_EUNSUP (grid above 96 points). */
int32_t paro_truncated_gradient_workspace_bytes(paro_plan plan, int32_t nb, int32_t n_outer, int32_t n_cg,
                                                size_t *bytes);
int32_t paro_truncated_gradient(paro_plan plan, int32_t nb, const double *trial, int64_t ld, double sigma,
                                int32_t n_outer, int32_t n_cg, const double *weights, double *energy, double *dvloc,
                                double *dR, void *ws, size_t ws_bytes);

/* ---------------------------------------------------------------- building blocks */

/* Complex double GEMMs on the FP64 matrix cores, the products the hot
 * path is made of (all matrices column-major, dev memory, on stream s).
 * paro_zgemm_hn: C (M x N, ldc) = A^H B, A: K x M (lda), B: K x N (ldb);
 *   the K sum is split over work-groups into partial tiles held in ws
 *   (at least M * N * 16 bytes; more allows more splits) and reduced in a
 *   fixed order.
 * paro_zgemm_nn: C (M x N, ldc) = A B (+ C when accumulate), A: M x K,
 *   B: K x N. */
int32_t paro_zgemm_hn(paro_stream_t s, int32_t M, int32_t N, int64_t K, const double *A, int64_t lda,
                      const double *B, int64_t ldb, double *C, int64_t ldc, void *ws, size_t ws_bytes);
int32_t paro_zgemm_nn(paro_stream_t s, int64_t M, int32_t N, int32_t K, const double *A, int64_t lda,
                      const double *B, int64_t ldb, double *C, int64_t ldc, int32_t accumulate);

/* paro_zgemm_hn without a workspace, for callers that cannot allocate
 * device memory (code under graph capture, serving loops, harnesses that
 * forbid allocation): the split partial tiles go to a fixed 32 MiB device
 * array inside the library, one per device, held until the process ends.
 * Same product, arguments and layout as paro_zgemm_hn; s must be a stream
 * of the current device (or NULL).  The number of K splits depends on the
 * scratch size, so results can differ from paro_zgemm_hn's in rounding.
 * Calls on one device share the array: calls that overlap in time on one
 * device (different streams, or host threads) race and give wrong results.
 * The library calls no allocator here.  Errors: PARO_EINVAL (bad argument),
 * PARO_ESIZE (M * N * 16 bytes above 32 MiB), PARO_EHIP. */
int32_t paro_zgemm_hn_noalloc(paro_stream_t s, int32_t M, int32_t N, int64_t K, const double *A, int64_t lda,
                              const double *B, int64_t ldb, double *C, int64_t ldc);

/* The device Hermitian eigensolver of the Rayleigh-Ritz step: A (m x m,
 * column-major, dev, read only) = V diag(w) V^H, w ascending (dev
 * double[m]), V (dev complex m x m).  Householder tridiagonalisation,
 * bisection, inverse iteration, back-transformation.  m <= 1024.
 * ws: paro_heev_workspace_bytes(m). */
int32_t paro_heev_workspace_bytes(int32_t m, size_t *bytes);
int32_t paro_heev(paro_stream_t s, int32_t m, const double *A, double *w, double *V, void *ws, size_t ws_bytes);

#ifdef __cplusplus
}
#endif
#endif /* PARO_H */
