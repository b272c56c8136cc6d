// Drivers of the hot path: H psi, the source problems (Algorithm 1, step 3),
// Rayleigh-Ritz (step 4), residuals and the ParO outer loop (steps 1, 3-5;
// Algorithm 2 for the MParO I variant).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "paro_internal.h"

namespace paro {

hipError_t apply_full(const Plan &pl, const Workspace &w, int nb, const double2 *x, int64_t ld, double2 *out,
                      const double *shift)
{
    hipError_t e = launch_local_apply(pl, w, nb, x, ld, out, shift, nullptr, nullptr, false, nullptr, nullptr);
    if (e != hipSuccess || pl.nproj == 0) return e;
    // V_NL x = B D (B^H x)
    e = gemm_hn(pl.stream, pl.nproj, nb, pl.ng, pl.beta, pl.ldv, x, ld, w.P, pl.nproj, w.part, w.part_elems, pl.dkb,
                nullptr);
    if (e != hipSuccess) return e;
    return gemm_nn(pl.stream, pl.ng, nb, pl.nproj, pl.beta, pl.ldv, w.P, pl.nproj, out, ld, true);
}

// mode 0: the source problem of Algorithm 1 (from u = psi); 1: the
// correction equation of Algorithm 2 (from e = 0); 2: the projected
// correction equation of Algorithm 3 (from e = 0 in the complement of psi;
// r0, every z and every (H - sigma) p projected).
hipError_t source_solve(const Plan &pl, const Workspace &w, int nb, const double2 *psi, const double2 *hpsi,
                        int64_t ld, const double *eps, const double *shift, int ncg, double2 *u, int64_t ldu,
                        int32_t *band_flags, int mode)
{
    const double2 *proj = mode == 2 ? psi : nullptr;
    hipError_t e = launch_pcg_init(pl, w, nb, psi, hpsi, ld, eps, u, ldu, band_flags, mode >= 1, proj);
    double *pq_parts = w.dots + (size_t)DOT_PQ * nb * kMaxParts;
    for (int k = 1; k <= ncg && e == hipSuccess; ++k) {
        int npq = 0;
        // q = (H_loc + kin - sigma) p with p <- z + beta p
        e = launch_local_apply(pl, w, nb, w.z, pl.ldv, w.q, shift, w.p, w.sc + SC_BETA * nb, k == 1, pq_parts, &npq);
        if (e == hipSuccess && pl.nproj > 0) {
            e = gemm_hn(pl.stream, pl.nproj, nb, pl.ng, pl.beta, pl.ldv, w.p, pl.ldv, w.P, pl.nproj, w.part,
                        w.part_elems, pl.dkb, w.sc + SC_NLQ * nb);
            if (e == hipSuccess) e = gemm_nn(pl.stream, pl.ng, nb, pl.nproj, pl.beta, pl.ldv, w.P, pl.nproj, w.q,
                                             pl.ldv, true);
        }
        // p lies in the complement of psi, so p^H q is unchanged by the projection
        if (e == hipSuccess && proj) e = launch_project_out(pl, w, nb, psi, ld, w.q);
        if (e == hipSuccess) e = launch_pcg_update(pl, w, nb, u, ldu, npq, band_flags, proj, ld);
    }
    return e;
}

// The nonlocal part of a single-precision apply, out += V_NL x: FP32
// matrix-core products, or split-BF16 ones (bf16 true) with their operand
// pairs in scratch (cap bytes).
static hipError_t apply_nl_f32(const Plan &pl, const Workspace &w, int nb, const float2 *x, int64_t ld, float2 *out,
                               int64_t ldo, double *quad, bool bf16, void *scratch, size_t cap)
{
    if (pl.nproj == 0) return hipSuccess;
    if (bf16) {
        if (bf16_apply_scratch_bytes(pl, nb) > cap) return hipErrorInvalidValue;
        return apply_nl_bf16(pl, w, nb, x, ld, out, ldo, scratch, quad);
    }
    float2 *P = reinterpret_cast<float2 *>(w.P);
    hipError_t e = gemm_hn(pl.stream, pl.nproj, nb, pl.ng, pl.beta32, pl.ldv, x, ld, P, pl.nproj, w.part,
                           w.part_elems, pl.dkb, quad);
    if (e != hipSuccess) return e;
    return gemm_nn(pl.stream, pl.ng, nb, pl.nproj, pl.beta32, pl.ldv, P, pl.nproj, out, ldo, true);
}

// H x in single precision (FP32 plan tables; FP32 or split-BF16 matrix
// cores).  The split-BF16 operand pairs go to the W block of the
// workspace, which the single-precision apply does not use.
static hipError_t apply_full(const Plan &pl, const Workspace &w, int nb, int nbw, const float2 *x, int64_t ld,
                             float2 *out, const double *shift, bool bf16)
{
    hipError_t e = launch_local_apply(pl, w, nb, x, ld, out, shift, nullptr, nullptr, false, nullptr, nullptr);
    if (e != hipSuccess) return e;
    return apply_nl_f32(pl, w, nb, x, ld, out, ld, nullptr, bf16, w.W, sizeof(double2) * 2 * (size_t)nbw * pl.ldv);
}

// Mixed-precision source problems: the correction d = u - psi solves
// (H - sigma) d = eps psi - H psi (the same problem as source_solve, moved
// by the FP64 psi), by n_cg PCG steps from d = 0 with FP32 vectors, FP32
// applies of H and FP64 scalars; the right-hand side is formed in FP64 from
// the carried FP64 H psi, and u = psi + d (or u = d when correction) is
// written in FP64.  The FP64 Rayleigh-Ritz that follows acts as the
// refinement: the FP32 error is relative to d, which vanishes as the bands
// converge.
// With bf16 the projector products run as split-BF16 products, their
// operand pairs in the W block past d (the correction, in its first
// quarter).
static hipError_t source_solve_mixed(const Plan &pl, const Workspace &w, int nb, const double2 *psi,
                                     const double2 *hpsi, int64_t ld, const double *eps, const double *shift, int ncg,
                                     double2 *u, int64_t ldu, int32_t *band_flags, bool correction, bool bf16)
{
    hipError_t e = launch_pcg_init_mixed(pl, w, nb, psi, hpsi, ld, eps, band_flags);
    double *pq_parts = w.dots + (size_t)DOT_PQ * nb * kMaxParts;
    void *scratch = reinterpret_cast<char *>(w.W) + sizeof(float2) * (size_t)nb * pl.ldv;
    const size_t cap = sizeof(float2) * 3 * (size_t)nb * pl.ldv;
    for (int k = 1; k <= ncg && e == hipSuccess; ++k) {
        int npq = 0;
        e = launch_local_apply(pl, w, nb, w.z32, pl.ldv, w.q32, shift, w.p32, w.sc + SC_BETA * nb, k == 1, pq_parts,
                               &npq);
        if (e == hipSuccess)
            e = apply_nl_f32(pl, w, nb, w.p32, pl.ldv, w.q32, pl.ldv, w.sc + SC_NLQ * nb, bf16, scratch, cap);
        if (e == hipSuccess) e = launch_pcg_update_mixed(pl, w, nb, npq, band_flags);
    }
    if (e == hipSuccess) e = launch_finish_correction(pl, w, nb, correction ? nullptr : psi, ld, u, ldu);
    return e;
}

hipError_t rayleigh_ritz(const Plan &pl, const Workspace &w, int m, int nkeep, const double2 *U, const double2 *W,
                         int64_t ld, double *eps, double2 *psi, double2 *hpsi, int64_t ldo)
{
    hipError_t e = gemm_hn(pl.stream, m, m, pl.ng, U, ld, U, ld, w.gram, m, w.part, w.part_elems, nullptr, nullptr);
    if (e == hipSuccess)
        e = gemm_hn(pl.stream, m, m, pl.ng, U, ld, W, ld, w.gram + (size_t)m * m, m, w.part, w.part_elems, nullptr,
                    nullptr);
    if (e == hipSuccess) e = launch_rr_dense(pl, w, m, nkeep, eps, w.dense[4]);
    if (e == hipSuccess) e = gemm_nn(pl.stream, pl.ng, nkeep, m, U, ld, w.dense[4], m, psi, ldo, false);
    if (e == hipSuccess) e = gemm_nn(pl.stream, pl.ng, nkeep, m, W, ld, w.dense[4], m, hpsi, ldo, false);
    return e;
}

}  // namespace paro

using namespace paro;

#define PARO_CHECK_LAUNCH(expr)                                                  \
    do {                                                                         \
        hipError_t _e = (expr);                                                  \
        if (_e != hipSuccess) {                                                  \
            set_error(std::string("kernel launch: ") + hipGetErrorString(_e));   \
            return PARO_EHIP;                                                    \
        }                                                                        \
    } while (0)

// Largest Rayleigh-Ritz subspace of the device dense path (m x m eigensolve).
constexpr int kMaxIterBands = 1024;

static int32_t check_ws(const Plan &pl, int nb, void *ws, size_t ws_bytes)
{
    if (!ws) {
        set_error("workspace is NULL");
        return PARO_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(ws) % 256) {
        set_error("workspace must be 256-byte aligned");
        return PARO_EINVAL;
    }
    if (ws_bytes < workspace_bytes(pl, nb)) {
        set_error("workspace smaller than paro_workspace_bytes");
        return PARO_ESIZE;
    }
    return PARO_OK;
}

extern "C" {

int32_t paro_apply_h(paro_plan plan, int32_t nb, const double *psi, int64_t ld, const double *shift, double *hpsi,
                     void *ws, size_t ws_bytes)
{
    if (!plan || nb <= 0 || !psi || !hpsi) {
        set_error("paro_apply_h: bad argument");
        return PARO_EINVAL;
    }
    const Plan &pl = plan->pl;
    if (ld < pl.ng) {
        set_error("paro_apply_h: ld < n_g");
        return PARO_EINVAL;
    }
    const int nbw = (nb + 1) / 2;  // workspace of nbw bands serves applies on 2 nbw bands
    int32_t rc = check_ws(pl, nbw, ws, ws_bytes);
    if (rc) return rc;
    Workspace w = carve_workspace(pl, nbw, ws);
    PARO_CHECK_LAUNCH(apply_full(pl, w, nb, (const double2 *)psi, ld, (double2 *)hpsi, shift));
    return PARO_OK;
}

int32_t paro_density_workspace_bytes(paro_plan plan, int32_t nb, size_t *bytes)
{
    if (!plan || nb <= 0 || !bytes) {
        set_error("paro_density_workspace_bytes: bad argument");
        return PARO_EINVAL;
    }
    *bytes = density_workspace_bytes(plan->pl, nb, nullptr);
    return PARO_OK;
}

int32_t paro_density(paro_plan plan, int32_t nb, const double *psi, int64_t ld, const double *weights, double *rho,
                     void *ws, size_t ws_bytes)
{
    if (!plan || nb <= 0 || !psi || !rho || !ws) {
        set_error("paro_density: bad argument");
        return PARO_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(ws) % 256) {
        set_error("paro_density: workspace must be 256-byte aligned");
        return PARO_EINVAL;
    }
    const Plan &pl = plan->pl;
    if (ld < pl.ng) {
        set_error("paro_density: ld < n_g");
        return PARO_EINVAL;
    }
    if (big_grid(pl.grid[0])) {
        set_error("paro_density: grids above 96 points are not supported");
        return PARO_EUNSUP;
    }
    size_t off = 0;
    if (ws_bytes < density_workspace_bytes(pl, nb, &off)) {
        set_error("paro_density: workspace smaller than paro_density_workspace_bytes");
        return PARO_ESIZE;
    }
    char *base = static_cast<char *>(ws);
    PARO_CHECK_LAUNCH(launch_density(pl, reinterpret_cast<double2 *>(base), reinterpret_cast<double *>(base + off),
                                     nb, (const double2 *)psi, ld, weights, rho));
    return PARO_OK;
}

int32_t paro_projector_gradient_workspace_bytes(paro_plan plan, int32_t nb, size_t *bytes)
{
    if (!plan || nb <= 0 || !bytes) {
        set_error("paro_projector_gradient_workspace_bytes: bad argument");
        return PARO_EINVAL;
    }
    proj_grad_workspace(plan->pl, nb, nullptr, bytes);
    return PARO_OK;
}

int32_t paro_projector_gradient(paro_plan plan, int32_t nb, const double *psi, int64_t ld, const double *weights,
                                double *dd, double *dR, void *ws, size_t ws_bytes)
{
    if (!plan || nb <= 0 || !psi || !dd || !dR || !ws) {
        set_error("paro_projector_gradient: bad argument");
        return PARO_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(ws) % 256) {
        set_error("paro_projector_gradient: workspace must be 256-byte aligned");
        return PARO_EINVAL;
    }
    const Plan &pl = plan->pl;
    if (ld < pl.ng) {
        set_error("paro_projector_gradient: ld < n_g");
        return PARO_EINVAL;
    }
    size_t need = 0;
    ProjGradWs w = proj_grad_workspace(pl, nb, ws, &need);
    if (ws_bytes < need) {
        set_error("paro_projector_gradient: workspace smaller than paro_projector_gradient_workspace_bytes");
        return PARO_ESIZE;
    }
    PARO_CHECK_LAUNCH(launch_projector_gradient(pl, w, nb, (const double2 *)psi, ld, weights, dd, dR));
    return PARO_OK;
}

static int32_t apply_f32_entry(const char *name, paro_plan plan, int32_t nb, const float *psi, int64_t ld,
                               const double *shift, float *hpsi, void *ws, size_t ws_bytes, bool bf16)
{
    if (!plan || nb <= 0 || !psi || !hpsi) {
        set_error(std::string(name) + ": bad argument");
        return PARO_EINVAL;
    }
    const Plan &pl = plan->pl;
    if (ld < pl.ng) {
        set_error(std::string(name) + ": ld < n_g");
        return PARO_EINVAL;
    }
    const int nbw = (nb + 1) / 2;
    int32_t rc = check_ws(pl, nbw, ws, ws_bytes);
    if (rc) return rc;
    Workspace w = carve_workspace(pl, nbw, ws);
    PARO_CHECK_LAUNCH(apply_full(pl, w, nb, nbw, (const float2 *)psi, ld, (float2 *)hpsi, shift, bf16));
    return PARO_OK;
}

int32_t paro_apply_h_f32(paro_plan plan, int32_t nb, const float *psi, int64_t ld, const double *shift, float *hpsi,
                         void *ws, size_t ws_bytes)
{
    return apply_f32_entry("paro_apply_h_f32", plan, nb, psi, ld, shift, hpsi, ws, ws_bytes, false);
}

int32_t paro_apply_h_f32_bf16(paro_plan plan, int32_t nb, const float *psi, int64_t ld, const double *shift,
                              float *hpsi, void *ws, size_t ws_bytes)
{
    return apply_f32_entry("paro_apply_h_f32_bf16", plan, nb, psi, ld, shift, hpsi, ws, ws_bytes, true);
}

int32_t paro_source_solve_mixed(paro_plan plan, int32_t nb, const double *psi, const double *hpsi, int64_t ld,
                                const double *eps, const double *shift, int32_t n_cg, double *u,
                                int32_t *band_flags, void *ws, size_t ws_bytes)
{
    if (!plan || nb <= 0 || !psi || !hpsi || !eps || !shift || !u || n_cg < 0) {
        set_error("paro_source_solve_mixed: bad argument");
        return PARO_EINVAL;
    }
    const Plan &pl = plan->pl;
    if (ld < pl.ng) {
        set_error("paro_source_solve_mixed: ld < n_g");
        return PARO_EINVAL;
    }
    int32_t rc = check_ws(pl, nb, ws, ws_bytes);
    if (rc) return rc;
    Workspace w = carve_workspace(pl, nb, ws);
    PARO_CHECK_LAUNCH(source_solve_mixed(pl, w, nb, (const double2 *)psi, (const double2 *)hpsi, ld, eps, shift,
                                         n_cg, (double2 *)u, ld, band_flags, false, false));
    return PARO_OK;
}

int32_t paro_source_solve(paro_plan plan, int32_t nb, const double *psi, const double *hpsi, int64_t ld,
                          const double *eps, const double *shift, int32_t n_cg, double *u, int32_t *band_flags,
                          void *ws, size_t ws_bytes)
{
    if (!plan || nb <= 0 || !psi || !hpsi || !eps || !shift || !u || n_cg < 0) {
        set_error("paro_source_solve: bad argument");
        return PARO_EINVAL;
    }
    const Plan &pl = plan->pl;
    if (ld < pl.ng) {
        set_error("paro_source_solve: ld < n_g");
        return PARO_EINVAL;
    }
    int32_t rc = check_ws(pl, nb, ws, ws_bytes);
    if (rc) return rc;
    Workspace w = carve_workspace(pl, nb, ws);
    PARO_CHECK_LAUNCH(source_solve(pl, w, nb, (const double2 *)psi, (const double2 *)hpsi, ld, eps, shift, n_cg,
                                   (double2 *)u, ld, band_flags));
    return PARO_OK;
}

int32_t paro_rayleigh_ritz(paro_plan plan, int32_t m, int32_t n_keep, const double *U, const double *W, int64_t ld,
                           double *eps, double *psi, double *hpsi, void *ws, size_t ws_bytes)
{
    if (!plan || m <= 0 || n_keep <= 0 || n_keep > m || !U || !W || !eps || !psi || !hpsi || m > 1024) {
        set_error("paro_rayleigh_ritz: bad argument (1 <= n_keep <= m <= 1024)");
        return PARO_EINVAL;
    }
    const Plan &pl = plan->pl;
    if (ld < pl.ng) {
        set_error("paro_rayleigh_ritz: ld < n_g");
        return PARO_EINVAL;
    }
    if (m > kMaxIterBands) {
        set_error("paro_rayleigh_ritz: m above " + std::to_string(kMaxIterBands));
        return PARO_EUNSUP;
    }
    const int nbw = (m + 1) / 2;
    int32_t rc = check_ws(pl, nbw, ws, ws_bytes);
    if (rc) return rc;
    Workspace w = carve_workspace(pl, nbw, ws);
    PARO_CHECK_LAUNCH(rayleigh_ritz(pl, w, m, n_keep, (const double2 *)U, (const double2 *)W, ld, eps,
                                    (double2 *)psi, (double2 *)hpsi, ld));
    return PARO_OK;
}

int32_t paro_residual_norms(paro_plan plan, int32_t nb, const double *psi, const double *hpsi, int64_t ld,
                            const double *eps, double *res, void *ws, size_t ws_bytes)
{
    if (!plan || nb <= 0 || !psi || !hpsi || !eps || !res) {
        set_error("paro_residual_norms: bad argument");
        return PARO_EINVAL;
    }
    const Plan &pl = plan->pl;
    if (ld < pl.ng) {
        set_error("paro_residual_norms: ld < n_g");
        return PARO_EINVAL;
    }
    int32_t rc = check_ws(pl, nb, ws, ws_bytes);
    if (rc) return rc;
    Workspace w = carve_workspace(pl, nb, ws);
    PARO_CHECK_LAUNCH(launch_residuals(pl, w, nb, (const double2 *)psi, (const double2 *)hpsi, ld, eps, res));
    return PARO_OK;
}

int32_t paro_shift_lower_bound(paro_plan plan, double *sigma_dev, void *ws, size_t ws_bytes)
{
    if (!plan || !sigma_dev) {
        set_error("paro_shift_lower_bound: bad argument");
        return PARO_EINVAL;
    }
    const Plan &pl = plan->pl;
    const int nbw = pl.nproj > 1 ? (pl.nproj + 1) / 2 : 1;
    int32_t rc = check_ws(pl, nbw, ws, ws_bytes);
    if (rc) return rc;
    Workspace w = carve_workspace(pl, nbw, ws);
    PARO_CHECK_LAUNCH(launch_shift_bound(pl, w, sigma_dev));
    return PARO_OK;
}

namespace {

// One problem of paro_iterate / paro_iterate_batch: its plan, block,
// workspace and options, and the host-side state of its outer loop.
struct CellRun {
    const Plan *pl = nullptr;
    Workspace w{};
    int nb = 0;
    double2 *psi = nullptr, *hpsi = nullptr;
    int64_t ld = 0;
    double *eps = nullptr, *sigma = nullptr, *stats = nullptr;
    paro_iter_opts o{};
    int32_t *conv = nullptr;  // device flag: converged to tol_res
    int32_t *n_done = nullptr;
    bool active = true, solve = false;
    // pinned host copies of the device values the loop decides on, so that
    // the copies are asynchronous and the cells' work is all in flight
    int32_t *hconv = nullptr;
    double *scur = nullptr;
    int32_t *hflags = nullptr;
};

// Page-locked host memory for the per-cell decision values, freed on scope exit.
struct PinnedHost {
    void *p = nullptr;
    ~PinnedHost()
    {
        if (p) (void)hipHostFree(p);
    }
};

int32_t prepare_cell(paro_plan plan, int32_t nb, double *psi, double *hpsi, int64_t ld, double *eps, double *sigma,
                     const paro_iter_opts *opts, double *stats, void *ws, size_t ws_bytes, int32_t *n_done,
                     CellRun &c)
{
    if (!plan || nb <= 0 || !psi || !hpsi || !eps || !sigma || !opts || opts->n_outer < 0 || opts->n_cg < 0 ||
        nb > kMaxIterBands ||
        (opts->variant != PARO_VARIANT_PARO && opts->variant != PARO_VARIANT_MPARO1 &&
         opts->variant != PARO_VARIANT_MPARO2) ||
        (opts->shift_mode != PARO_SHIFT_FIXED && opts->shift_mode != PARO_SHIFT_ADAPTIVE) ||
        (opts->precision != PARO_PREC_FP64 && opts->precision != PARO_PREC_MIXED &&
         opts->precision != PARO_PREC_MIXED_BF16)) {
        set_error("paro_iterate: bad argument");
        return PARO_EINVAL;
    }
    const Plan &pl = plan->pl;
    if (ld < pl.ng) {
        set_error("paro_iterate: ld < n_g");
        return PARO_EINVAL;
    }
    if (opts->variant != PARO_VARIANT_PARO && 2 * nb > kMaxIterBands) {
        set_error("paro_iterate: MParO runs Rayleigh-Ritz on 2 nb vectors, at most " +
                  std::to_string(kMaxIterBands));
        return PARO_EUNSUP;
    }
    if (opts->variant == PARO_VARIANT_MPARO2 && opts->precision != PARO_PREC_FP64) {
        set_error("paro_iterate: MParO II runs in FP64 only");
        return PARO_EUNSUP;
    }
    int32_t rc = check_ws(pl, nb, ws, ws_bytes);
    if (rc) return rc;
    c.pl = &pl;
    c.w = carve_workspace(pl, nb, ws);
    c.nb = nb;
    c.psi = (double2 *)psi;
    c.hpsi = (double2 *)hpsi;
    c.ld = ld;
    c.eps = eps;
    c.sigma = sigma;
    c.stats = stats;
    c.o = *opts;
    c.conv = reinterpret_cast<int32_t *>(c.w.scal + 1);
    c.n_done = n_done;
    if (n_done) *n_done = 0;
    return PARO_OK;
}

// Events, freed on scope exit.
struct EventSet {
    std::vector<hipEvent_t> ev;
    ~EventSet()
    {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

enum class Phase { Start, WaitConv, WaitSolve, Done };

// Enqueue the source problems of the cell's current iteration (Algorithm 1
// step 3, or the correction equation of Algorithms 2 and 3).
hipError_t enqueue_solve(CellRun &c)
{
    const Plan &pl = *c.pl;
    Workspace &w = c.w;
    const int64_t lv = pl.ldv;
    const bool mparo = c.o.variant != PARO_VARIANT_PARO;
    double2 *Ut = mparo ? w.U + (size_t)c.nb * lv : w.U;  // u (Algorithm 1) or e (Algorithms 2, 3)
    if (c.o.precision != PARO_PREC_FP64)
        return source_solve_mixed(pl, w, c.nb, c.psi, c.hpsi, c.ld, c.eps, w.sig_all, c.o.n_cg, Ut, lv,
                                  w.iflags + c.nb, mparo, c.o.precision == PARO_PREC_MIXED_BF16);
    return source_solve(pl, w, c.nb, c.psi, c.hpsi, c.ld, c.eps, w.sig_all, c.o.n_cg, Ut, lv, w.iflags + c.nb,
                        c.o.variant);
}

// Enqueue Rayleigh-Ritz (steps 4), residuals, the next shift and the
// statistics row of iteration it (step 5).
hipError_t enqueue_finish(CellRun &c, int it)
{
    const Plan &pl = *c.pl;
    Workspace &w = c.w;
    const int64_t lv = pl.ldv;
    const int nb = c.nb;
    hipError_t e;
    if (c.o.variant != PARO_VARIANT_PARO) {
        // span{psi, e/|e|}, e from the correction equation (Algorithms 2, 3)
        double2 *Ut = w.U + (size_t)nb * lv;
        if ((e = launch_normalize_bands(pl, w, nb, Ut, lv)) != hipSuccess) return e;
        if ((e = launch_copy_bands(pl.stream, nb, pl.ng, c.psi, c.ld, w.U, lv)) != hipSuccess) return e;
        if ((e = launch_copy_bands(pl.stream, nb, pl.ng, c.hpsi, c.ld, w.W, lv)) != hipSuccess) return e;
        if ((e = apply_full(pl, w, nb, Ut, lv, w.W + (size_t)nb * lv, nullptr)) != hipSuccess) return e;
        if ((e = rayleigh_ritz(pl, w, 2 * nb, nb, w.U, w.W, lv, c.eps, c.psi, c.hpsi, c.ld)) != hipSuccess) return e;
    } else {
        if ((e = apply_full(pl, w, nb, w.U, lv, w.W, nullptr)) != hipSuccess) return e;
        if ((e = rayleigh_ritz(pl, w, nb, nb, w.U, w.W, lv, c.eps, c.psi, c.hpsi, c.ld)) != hipSuccess) return e;
    }
    const int row = 2 * nb + 2;
    if ((e = launch_residuals(pl, w, nb, c.psi, c.hpsi, c.ld, c.eps, w.res)) != hipSuccess) return e;
    return launch_bookkeeping(pl, nb, c.o, c.eps, w.res, w.sig_all, c.sigma,
                              c.stats ? c.stats + (size_t)(it + 1) * row : nullptr, c.conv);
}

// The outer loop of Algorithm 1 (or 2, 3) for every cell.  Each cell's
// kernels go to its plan's stream.  The host decisions of an iteration (the
// convergence test, the negative-curvature retry of the adaptive shift) read
// small device values copied into pinned host memory behind an event; the
// host polls the cells' events and moves each cell on as soon as its own
// values have arrived, so that no cell waits for another and the GPU always
// holds the work of every cell that is not waiting.  A cell's sequence of
// launches is the same as when it runs alone.
int32_t run_cells(std::vector<CellRun> &cells)
{
    // Host decisions exist only with a tolerance or the adaptive shift;
    // without them the loop only enqueues kernels (no host memory, events or
    // waits), so a caller can capture it into a graph.
    bool decide = false;
    for (const CellRun &c : cells) decide = decide || c.o.tol_res > 0.0 || c.o.shift_mode == PARO_SHIFT_ADAPTIVE;
    const int n = (int)cells.size();
    PinnedHost host;
    EventSet events;
    if (decide) {
        // per cell: sigma (double), the convergence flag, the band flags; 8-byte blocks
        auto block = [](const CellRun &c) { return sizeof(double) + (sizeof(int32_t) * (2 + c.nb) + 7) / 8 * 8; };
        size_t bytes = 0;
        for (const CellRun &c : cells) bytes += block(c);
        PARO_HIP_TRY(hipHostMalloc(&host.p, bytes, hipHostMallocDefault));
        char *q = static_cast<char *>(host.p);
        for (CellRun &c : cells) {
            c.scur = reinterpret_cast<double *>(q);
            c.hconv = reinterpret_cast<int32_t *>(q + sizeof(double));
            c.hflags = c.hconv + 2;
            q += block(c);
        }
        events.ev.assign(n, nullptr);
        for (int i = 0; i < n; ++i) PARO_HIP_TRY(hipEventCreateWithFlags(&events.ev[i], hipEventDisableTiming));
    }
    for (CellRun &c : cells) {
        const Plan &pl = *c.pl;
        Workspace &w = c.w;
        const int64_t lv = pl.ldv;
        if (c.o.initial_rr) {
            PARO_CHECK_LAUNCH(launch_copy_bands(pl.stream, c.nb, pl.ng, c.psi, c.ld, w.U, lv));
            PARO_CHECK_LAUNCH(apply_full(pl, w, c.nb, w.U, lv, w.W, nullptr));
            PARO_CHECK_LAUNCH(rayleigh_ritz(pl, w, c.nb, c.nb, w.U, w.W, lv, c.eps, c.psi, c.hpsi, c.ld));
        }
        PARO_CHECK_LAUNCH(launch_residuals(pl, w, c.nb, c.psi, c.hpsi, c.ld, c.eps, w.res));
        PARO_CHECK_LAUNCH(launch_bookkeeping(pl, c.nb, c.o, c.eps, w.res, w.sig_all, c.sigma, c.stats, c.conv));
    }
    std::vector<Phase> phase(n, Phase::Start);
    std::vector<int> iter(n, 0), attempt(n, 0);
    // solve, then either wait for the curvature flags or finish the iteration
    auto solve_step = [&](int i) -> int32_t {
        CellRun &c = cells[i];
        PARO_CHECK_LAUNCH(enqueue_solve(c));
        if (c.o.shift_mode == PARO_SHIFT_ADAPTIVE) {
            PARO_HIP_TRY(hipMemcpyAsync(c.hflags, c.w.iflags + c.nb, sizeof(int32_t) * c.nb, hipMemcpyDeviceToHost,
                                        c.pl->stream));
            PARO_HIP_TRY(hipMemcpyAsync(c.scur, c.sigma, sizeof(double), hipMemcpyDeviceToHost, c.pl->stream));
            PARO_HIP_TRY(hipEventRecord(events.ev[i], c.pl->stream));
            phase[i] = Phase::WaitSolve;
            return PARO_OK;
        }
        PARO_CHECK_LAUNCH(enqueue_finish(c, iter[i]));
        if (c.n_done) *c.n_done = iter[i] + 1;
        ++iter[i];
        phase[i] = Phase::Start;
        return PARO_OK;
    };
    for (;;) {
        bool left = false, moved = false;
        int waiting = -1;
        for (int i = 0; i < n; ++i) {
            CellRun &c = cells[i];
            if (phase[i] == Phase::Done) continue;
            left = true;
            if (phase[i] == Phase::WaitConv || phase[i] == Phase::WaitSolve) {
                const hipError_t q = hipEventQuery(events.ev[i]);
                if (q == hipErrorNotReady) {
                    if (waiting < 0) waiting = i;
                    continue;
                }
                PARO_HIP_TRY(q);
            }
            moved = true;
            int32_t rc = PARO_OK;
            switch (phase[i]) {
            case Phase::Start:
                if (iter[i] >= c.o.n_outer) {
                    phase[i] = Phase::Done;
                } else if (c.o.tol_res > 0.0) {
                    PARO_HIP_TRY(
                        hipMemcpyAsync(c.hconv, c.conv, sizeof(int32_t), hipMemcpyDeviceToHost, c.pl->stream));
                    PARO_HIP_TRY(hipEventRecord(events.ev[i], c.pl->stream));
                    phase[i] = Phase::WaitConv;
                } else {
                    attempt[i] = 0;
                    rc = solve_step(i);
                }
                break;
            case Phase::WaitConv:
                if (*c.hconv) {
                    phase[i] = Phase::Done;
                } else {
                    attempt[i] = 0;
                    rc = solve_step(i);
                }
                break;
            case Phase::WaitSolve: {
                bool neg = false;
                for (int b = 0; b < c.nb; ++b) neg = neg || (c.hflags[b] & PARO_F_NEGCURV);
                if (neg && *c.scur != c.o.sigma_lb && attempt[i] == 0) {
                    // negative curvature: solve again with sigma_lb
                    paro_iter_opts fixed = c.o;
                    fixed.shift_mode = PARO_SHIFT_FIXED;
                    fixed.tol_res = 0.0;
                    PARO_CHECK_LAUNCH(launch_bookkeeping(*c.pl, c.nb, fixed, c.eps, c.w.res, c.w.sig_all, c.sigma,
                                                         nullptr, c.conv));
                    attempt[i] = 1;
                    rc = solve_step(i);
                } else {
                    PARO_CHECK_LAUNCH(enqueue_finish(c, iter[i]));
                    if (c.n_done) *c.n_done = iter[i] + 1;
                    ++iter[i];
                    phase[i] = Phase::Start;
                }
                break;
            }
            case Phase::Done:
                break;
            }
            if (rc) return rc;
        }
        if (!left) break;
        // every cell is waiting for the GPU: block on the first one rather
        // than spin (the others' work continues meanwhile)
        if (!moved && waiting >= 0) PARO_HIP_TRY(hipEventSynchronize(events.ev[waiting]));
    }
    return PARO_OK;
}

// Whether a batch can run its source problems as grouped launches: FP64
// Algorithm 1 or 2 on grids with grouped kernels, more than one cell.
bool groupable(const std::vector<CellRun> &cells)
{
    if (cells.size() < 2) return false;
    for (const CellRun &c : cells)
        if ((c.o.precision != PARO_PREC_FP64 && c.o.precision != PARO_PREC_MIXED) ||
            c.o.precision != cells[0].o.precision || c.o.variant == PARO_VARIANT_MPARO2 ||
            !grouped_grid(c.pl->grid[0]) || c.nb > kGroupChunks * kMaxBandsPerChunk)
            return false;
    return true;
}

// The source problems of the given cells (Algorithm 1 step 3, or the
// correction equation of Algorithm 2) as grouped launches on stream s: per
// PCG step one launch per kernel and FFT length for all cells, each cell's
// work exactly that of its own source_solve.
extern "C++" {
// C2 = float2: the mixed-precision solve of the correction (FP32 vectors,
// FP32 matrix-core products), ending with u = psi + d (or d) per cell.
template <class C2>
hipError_t source_solve_grouped(hipStream_t s, const std::vector<GroupCell> &gc, const std::vector<int> &ncg,
                                const std::vector<const CellRun *> &cr)
{
    const int n = (int)gc.size();
    hipError_t e = launch_pcg_init_grouped<C2>(s, gc.data(), n);
    int kmax = 0;
    for (int k : ncg) kmax = std::max(kmax, k);
    std::vector<GroupCell> sub;
    for (int k = 1; k <= kmax && e == hipSuccess; ++k) {
        sub.clear();
        for (int i = 0; i < n; ++i)
            if (ncg[i] >= k) sub.push_back(gc[i]);
        const int m = (int)sub.size();
        e = launch_local_apply_grouped<C2>(s, sub.data(), m, k == 1);
        if (e == hipSuccess) e = launch_nonlocal_grouped<C2>(s, sub.data(), m);
        if (e == hipSuccess) e = launch_pcg_update_grouped<C2>(s, sub.data(), m);
    }
    if constexpr (sizeof(C2) == 8) {
        for (int i = 0; i < n && e == hipSuccess; ++i) {
            const CellRun &c = *cr[i];
            const bool mparo = c.o.variant != PARO_VARIANT_PARO;
            double2 *Ut = mparo ? c.w.U + (size_t)c.nb * c.pl->ldv : c.w.U;
            Plan pl = *c.pl;
            pl.stream = s;
            e = launch_finish_correction(pl, c.w, c.nb, mparo ? nullptr : c.psi, c.ld, Ut, c.pl->ldv);
        }
    }
    return e;
}

}  // extern "C++"

// Steps 4-5 of Algorithm 1 for the given cells as grouped launches, each
// cell's work that of its enqueue_finish: W = H U, Rayleigh-Ritz at m = nb
// (Gram products, the dense eigenproblem, the rotations), residuals, the
// next shift and the statistics row of iteration it.
hipError_t finish_grouped(hipStream_t s, const std::vector<GroupCell> &gc, int it)
{
    const int n = (int)gc.size();
    hipError_t e = launch_finish_local_grouped(s, gc.data(), n);
    std::vector<HnRef<double2>> hv;
    std::vector<NnRef<double2>> nv;
    for (const GroupCell &c : gc)
        if (c.pl->nproj > 0) {
            hv.push_back(HnRef<double2>{&c.dev->fin.nl_hn, &c.host->fin.nl_hn, &c.dev->fin.nl_red});
            nv.push_back(NnRef<double2>{&c.dev->fin.nl_nn, &c.host->fin.nl_nn});
        }
    if (e == hipSuccess) e = launch_hn_grouped<double2>(s, hv.data(), (int)hv.size());
    if (e == hipSuccess) e = launch_nn_grouped<double2>(s, nv.data(), (int)nv.size());
    // S = U^H U, then H_s = U^H W (each cell's split partials are reused)
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        hv.clear();
        for (const GroupCell &c : gc)
            hv.push_back(k == 0 ? HnRef<double2>{&c.dev->fin.s_hn, &c.host->fin.s_hn, &c.dev->fin.s_red}
                                : HnRef<double2>{&c.dev->fin.h_hn, &c.host->fin.h_hn, &c.dev->fin.h_red});
        e = launch_hn_grouped<double2>(s, hv.data(), n);
    }
    if (e == hipSuccess) e = launch_rr_dense_grouped(s, gc.data(), n);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        nv.clear();
        for (const GroupCell &c : gc)
            nv.push_back(k == 0 ? NnRef<double2>{&c.dev->fin.rot_psi, &c.host->fin.rot_psi}
                                : NnRef<double2>{&c.dev->fin.rot_hpsi, &c.host->fin.rot_hpsi});
        e = launch_nn_grouped<double2>(s, nv.data(), n);
    }
    if (e == hipSuccess) e = launch_residuals_grouped(s, gc.data(), n);
    if (e == hipSuccess) e = launch_bookkeeping_grouped(s, gc.data(), n, it);
    return e;
}

// The outer loop of run_cells with the cells in lockstep: every outer
// iteration, the source problems of all cells still iterating run as
// grouped launches on the first such cell's stream (ordered against each
// cell's own stream by events), then each cell's Rayleigh-Ritz, residuals
// and shift run on its own stream as before, side by side.  The host takes
// the same decisions as run_cells, from the same device values, for all
// cells at once; each cell's device work is exactly that of its lone run.
int32_t run_cells_grouped(std::vector<CellRun> &cells)
{
    const int n = (int)cells.size();
    // Host decisions exist only with a tolerance or the adaptive shift.
    // They need, per cell, sigma, conv and the band flags in pinned host
    // memory.
    bool decide = false;
    for (const CellRun &c : cells) decide = decide || c.o.tol_res > 0.0 || c.o.shift_mode == PARO_SHIFT_ADAPTIVE;
    PinnedHost host;
    if (decide) {
        auto block = [](const CellRun &c) { return sizeof(double) + (sizeof(int32_t) * (2 + c.nb) + 7) / 8 * 8; };
        size_t bytes = 0;
        for (const CellRun &c : cells) bytes += block(c);
        PARO_HIP_TRY(hipHostMalloc(&host.p, bytes, hipHostMallocDefault));
        char *q = static_cast<char *>(host.p);
        for (CellRun &c : cells) {
            c.scur = reinterpret_cast<double *>(q);
            c.hconv = reinterpret_cast<int32_t *>(q + sizeof(double));
            c.hflags = c.hconv + 2;
            q += block(c);
        }
    }
    // host copies of the descriptors (uploaded through kernel arguments)
    std::vector<GroupCellDesc> hdesc(n);
    // Cells on one stream need no events to order the grouped launches
    // against their own work; with no host decision either, the call then
    // enqueues kernels only and can be captured into a graph.
    bool one_stream = true;
    for (const CellRun &c : cells) one_stream = one_stream && c.pl->stream == cells[0].pl->stream;
    EventSet events;
    if (decide || !one_stream) {
        events.ev.assign(n + 1, nullptr);
        for (int i = 0; i <= n; ++i) PARO_HIP_TRY(hipEventCreateWithFlags(&events.ev[i], hipEventDisableTiming));
    }
    hipEvent_t gev = events.ev.empty() ? nullptr : events.ev[n];
    std::vector<GroupCell> gc(n);
    std::vector<int> ncg(n);
    // steps 4-5 grouped too: Algorithm 1 with Rayleigh-Ritz at m = nb <= 92
    bool group_finish = true;
    for (const CellRun &c : cells)
        group_finish = group_finish && c.o.variant == PARO_VARIANT_PARO && rr_dense_groupable(c.nb);
    for (int i = 0; i < n; ++i) {
        CellRun &c = cells[i];
        const Plan &pl = *c.pl;
        Workspace &w = c.w;
        const int64_t lv = pl.ldv;
        const bool mparo = c.o.variant != PARO_VARIANT_PARO;
        double2 *Ut = mparo ? w.U + (size_t)c.nb * lv : w.U;
        GroupCellDesc &d = hdesc[i];
        std::memset(&d, 0, sizeof(d));
        const int npq = describe_local_apply(pl, w, c.nb, w.sig_all, d);
        describe_nonlocal(pl, w, c.nb, d);
        if (c.o.precision == PARO_PREC_MIXED)
            describe_pcg_mixed(pl, w, c.nb, c.psi, c.hpsi, c.ld, c.eps, w.iflags + c.nb, npq, d);
        else
            describe_pcg(pl, w, c.nb, c.psi, c.hpsi, c.ld, c.eps, Ut, lv, w.iflags + c.nb, mparo, npq, d);
        if (group_finish) {
            describe_finish_local(pl, w, c.nb, w.U, w.W, lv, d.fin);
            describe_finish_products(pl, w, c.nb, c.nb, w.U, w.W, lv, c.psi, c.hpsi, c.ld, d.fin);
            describe_rr_dense(pl, w, c.nb, c.nb, c.eps, w.dense[4], d.fin);
            describe_residuals(pl, w, c.nb, c.psi, c.hpsi, c.ld, c.eps, w.res, d.fin);
            describe_bookkeeping(pl, c.nb, c.o, c.eps, w.res, w.sig_all, c.sigma, c.stats, c.conv, d.fin);
        }
        PARO_CHECK_LAUNCH(upload_bytes(pl.stream, w.desc, &d, sizeof(d)));
        gc[i] = GroupCell{&pl, &w, c.nb, w.desc, &d};
        ncg[i] = c.o.n_cg;
        if (c.o.initial_rr) {
            PARO_CHECK_LAUNCH(launch_copy_bands(pl.stream, c.nb, pl.ng, c.psi, c.ld, w.U, lv));
            PARO_CHECK_LAUNCH(apply_full(pl, w, c.nb, w.U, lv, w.W, nullptr));
            PARO_CHECK_LAUNCH(rayleigh_ritz(pl, w, c.nb, c.nb, w.U, w.W, lv, c.eps, c.psi, c.hpsi, c.ld));
        }
        PARO_CHECK_LAUNCH(launch_residuals(pl, w, c.nb, c.psi, c.hpsi, c.ld, c.eps, w.res));
        PARO_CHECK_LAUNCH(launch_bookkeeping(pl, c.nb, c.o, c.eps, w.res, w.sig_all, c.sigma, c.stats, c.conv));
    }
    std::vector<int> iter(n, 0);
    std::vector<char> done(n, 0);
    std::vector<GroupCell> agc;
    std::vector<int> ancg, act;
    std::vector<const CellRun *> acr;
    const bool mixed = cells[0].o.precision == PARO_PREC_MIXED;
    for (;;) {
        // step 5 of the previous iteration: which cells go on
        bool wait = false;
        for (int i = 0; i < n; ++i) {
            CellRun &c = cells[i];
            if (done[i]) continue;
            if (iter[i] >= c.o.n_outer) {
                done[i] = 1;
            } else if (c.o.tol_res > 0.0) {
                PARO_HIP_TRY(hipMemcpyAsync(c.hconv, c.conv, sizeof(int32_t), hipMemcpyDeviceToHost, c.pl->stream));
                PARO_HIP_TRY(hipEventRecord(events.ev[i], c.pl->stream));
                wait = true;
            }
        }
        if (wait)
            for (int i = 0; i < n; ++i)
                if (!done[i] && cells[i].o.tol_res > 0.0) {
                    PARO_HIP_TRY(hipEventSynchronize(events.ev[i]));
                    if (*cells[i].hconv) done[i] = 1;
                }
        act.clear();
        for (int i = 0; i < n; ++i)
            if (!done[i]) act.push_back(i);
        if (act.empty()) break;
        // the grouped source problems, after each cell's own work so far
        hipStream_t gs = cells[act[0]].pl->stream;
        agc.clear();
        ancg.clear();
        acr.clear();
        for (int i : act) {
            if (!one_stream) {
                PARO_HIP_TRY(hipEventRecord(events.ev[i], cells[i].pl->stream));
                PARO_HIP_TRY(hipStreamWaitEvent(gs, events.ev[i], 0));
            }
            agc.push_back(gc[i]);
            ancg.push_back(ncg[i]);
            acr.push_back(&cells[i]);
        }
        if (mixed) PARO_CHECK_LAUNCH(source_solve_grouped<float2>(gs, agc, ancg, acr));
        else PARO_CHECK_LAUNCH(source_solve_grouped<double2>(gs, agc, ancg, acr));
        if (!one_stream) PARO_HIP_TRY(hipEventRecord(gev, gs));
        bool adaptive = false;
        for (int i : act) {
            CellRun &c = cells[i];
            if (!one_stream) PARO_HIP_TRY(hipStreamWaitEvent(c.pl->stream, gev, 0));
            if (c.o.shift_mode == PARO_SHIFT_ADAPTIVE) {
                PARO_HIP_TRY(hipMemcpyAsync(c.hflags, c.w.iflags + c.nb, sizeof(int32_t) * c.nb,
                                            hipMemcpyDeviceToHost, c.pl->stream));
                PARO_HIP_TRY(hipMemcpyAsync(c.scur, c.sigma, sizeof(double), hipMemcpyDeviceToHost, c.pl->stream));
                PARO_HIP_TRY(hipEventRecord(events.ev[i], c.pl->stream));
                adaptive = true;
            }
        }
        for (int i : act) {
            CellRun &c = cells[i];
            if (adaptive && c.o.shift_mode == PARO_SHIFT_ADAPTIVE) {
                PARO_HIP_TRY(hipEventSynchronize(events.ev[i]));
                bool neg = false;
                for (int b = 0; b < c.nb; ++b) neg = neg || (c.hflags[b] & PARO_F_NEGCURV);
                if (neg && *c.scur != c.o.sigma_lb) {
                    // negative curvature: the cell solves again alone with sigma_lb, as in run_cells
                    paro_iter_opts fixed = c.o;
                    fixed.shift_mode = PARO_SHIFT_FIXED;
                    fixed.tol_res = 0.0;
                    PARO_CHECK_LAUNCH(launch_bookkeeping(*c.pl, c.nb, fixed, c.eps, c.w.res, c.w.sig_all, c.sigma,
                                                         nullptr, c.conv));
                    PARO_CHECK_LAUNCH(enqueue_solve(c));
                    if (group_finish) {
                        PARO_HIP_TRY(hipEventRecord(events.ev[i], c.pl->stream));
                        PARO_HIP_TRY(hipStreamWaitEvent(gs, events.ev[i], 0));
                    }
                }
            }
            if (!group_finish) PARO_CHECK_LAUNCH(enqueue_finish(c, iter[i]));
        }
        if (group_finish) {
            // steps 4-5 of every cell as grouped launches on the same stream, then
            // each cell's stream waits for them
            PARO_CHECK_LAUNCH(finish_grouped(gs, agc, iter[act[0]]));
            if (!one_stream) {
                PARO_HIP_TRY(hipEventRecord(gev, gs));
                for (int i : act) PARO_HIP_TRY(hipStreamWaitEvent(cells[i].pl->stream, gev, 0));
            }
        }
        for (int i : act) {
            CellRun &c = cells[i];
            if (c.n_done) *c.n_done = iter[i] + 1;
            ++iter[i];
        }
    }
    return PARO_OK;
}

}  // namespace

int32_t paro_iterate(paro_plan plan, int32_t nb, double *psi, double *hpsi, int64_t ld, double *eps, double *sigma,
                     const paro_iter_opts *opts, double *stats, void *ws, size_t ws_bytes, int32_t *n_done)
{
    std::vector<CellRun> cells(1);
    int32_t rc = prepare_cell(plan, nb, psi, hpsi, ld, eps, sigma, opts, stats, ws, ws_bytes, n_done, cells[0]);
    if (rc) return rc;
    return run_cells(cells);
}

int32_t paro_iterate_batch(int32_t n_cells, const paro_plan *plans, const int32_t *nb, double *const *psi,
                           double *const *hpsi, const int64_t *ld, double *const *eps, double *const *sigma,
                           const paro_iter_opts *opts, double *const *stats, void *const *ws, const size_t *ws_bytes,
                           int32_t *n_done)
{
    if (n_cells <= 0 || !plans || !nb || !psi || !hpsi || !ld || !eps || !sigma || !opts || !ws || !ws_bytes) {
        set_error("paro_iterate_batch: bad argument");
        return PARO_EINVAL;
    }
    std::vector<CellRun> cells(n_cells);
    for (int i = 0; i < n_cells; ++i) {
        for (int k = 0; k < i; ++k)
            if (ws[k] == ws[i]) {
                set_error("paro_iterate_batch: cells " + std::to_string(k) + " and " + std::to_string(i) +
                          " share a workspace");
                return PARO_EINVAL;
            }
        int32_t rc = prepare_cell(plans[i], nb[i], psi[i], hpsi[i], ld[i], eps[i], sigma[i], &opts[i],
                                  stats ? stats[i] : nullptr, ws[i], ws_bytes[i], n_done ? n_done + i : nullptr,
                                  cells[i]);
        if (rc) {
            set_error("paro_iterate_batch: cell " + std::to_string(i) + ": " + paro_last_error());
            return rc;
        }
    }
    return groupable(cells) ? run_cells_grouped(cells) : run_cells(cells);
}

int32_t paro_zgemm_hn(paro_stream_t s, int32_t M, int32_t N, int64_t K, const double *A, int64_t lda,
                      const double *B, int64_t ldb, double *C, int64_t ldc, void *ws, size_t ws_bytes)
{
    if (M <= 0 || N <= 0 || K <= 0 || !A || !B || !C || !ws || lda < K || ldb < K || ldc < M) {
        set_error("paro_zgemm_hn: bad argument");
        return PARO_EINVAL;
    }
    if (ws_bytes < sizeof(double2) * (size_t)M * N) {
        set_error("paro_zgemm_hn: workspace smaller than M * N complex");
        return PARO_ESIZE;
    }
    PARO_CHECK_LAUNCH(gemm_hn(static_cast<hipStream_t>(s), M, N, K, (const double2 *)A, lda, (const double2 *)B, ldb,
                              (double2 *)C, ldc, (double2 *)ws, ws_bytes / sizeof(double2), nullptr, nullptr));
    return PARO_OK;
}

}  // extern "C"

namespace {

// Split-K partial tiles of paro_zgemm_hn_noalloc: a fixed device array
// instead of a caller workspace.  Each device that the library runs on
// holds its own copy until the process ends.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
__device__ __align__(256) double2 scratch[kNoAllocScratchBytes / sizeof(double2)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double2 *g_scratch_addr[kMaxDevices] = {};

// The device address of the current device's copy of scratch, looked up
// once per device (the array's name is a host-side stand-in, not a device
// address).
int32_t scratch_address(double2 **out)
{
    int dev = -1;
    PARO_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("paro_zgemm_hn_noalloc: device index out of range");
        return PARO_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        PARO_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("paro_zgemm_hn_noalloc: hipGetSymbolAddress returned NULL");
            return PARO_EHIP;
        }
        g_scratch_addr[dev] = static_cast<double2 *>(p);
    }
    *out = g_scratch_addr[dev];
    return PARO_OK;
}

}  // namespace

extern "C" {

int32_t paro_zgemm_hn_noalloc(paro_stream_t s, int32_t M, int32_t N, int64_t K, const double *A, int64_t lda,
                              const double *B, int64_t ldb, double *C, int64_t ldc)
{
    if (M <= 0 || N <= 0 || K <= 0 || !A || !B || !C || lda < K || ldb < K || ldc < M) {
        set_error("paro_zgemm_hn_noalloc: bad argument");
        return PARO_EINVAL;
    }
    if (sizeof(double2) * (size_t)M * (size_t)N > kNoAllocScratchBytes) {
        set_error("paro_zgemm_hn_noalloc: M * N * 16 bytes exceeds the " + std::to_string(kNoAllocScratchBytes) +
                  "-byte device scratch (use paro_zgemm_hn with a workspace)");
        return PARO_ESIZE;
    }
    double2 *part = nullptr;
    int32_t rc = scratch_address(&part);
    if (rc) return rc;
    // every split's partial tile is written in full before the reduce reads
    // it, so nothing from an earlier call needs clearing
    PARO_CHECK_LAUNCH(gemm_hn(static_cast<hipStream_t>(s), M, N, K, (const double2 *)A, lda, (const double2 *)B, ldb,
                              (double2 *)C, ldc, part, kNoAllocScratchBytes / sizeof(double2), nullptr, nullptr));
    return PARO_OK;
}

int32_t paro_zgemm_nn(paro_stream_t s, int64_t M, int32_t N, int32_t K, const double *A, int64_t lda,
                      const double *B, int64_t ldb, double *C, int64_t ldc, int32_t accumulate)
{
    if (M <= 0 || N <= 0 || K <= 0 || !A || !B || !C || lda < M || ldb < K || ldc < M) {
        set_error("paro_zgemm_nn: bad argument");
        return PARO_EINVAL;
    }
    PARO_CHECK_LAUNCH(gemm_nn(static_cast<hipStream_t>(s), M, N, K, (const double2 *)A, lda, (const double2 *)B, ldb,
                              (double2 *)C, ldc, accumulate != 0));
    return PARO_OK;
}

static size_t heev_bytes(int m)
{
    const size_t a = ((sizeof(double2) * (size_t)m * m) + 255) & ~(size_t)255;
    return a + sizeof(double) * dense_real_elems(m);
}

int32_t paro_heev_workspace_bytes(int32_t m, size_t *bytes)
{
    if (m <= 0 || m > 1024 || !bytes) {
        set_error("paro_heev_workspace_bytes: 1 <= m <= 1024");
        return PARO_EINVAL;
    }
    *bytes = heev_bytes(m);
    return PARO_OK;
}

int32_t paro_heev(paro_stream_t s, int32_t m, const double *A, double *w, double *V, void *ws, size_t ws_bytes)
{
    if (m <= 0 || m > 1024 || !A || !w || !V || !ws) {
        set_error("paro_heev: bad argument");
        return PARO_EINVAL;
    }
    if (ws_bytes < heev_bytes(m)) {
        set_error("paro_heev: workspace too small");
        return PARO_ESIZE;
    }
    Workspace wk{};
    char *base = static_cast<char *>(ws);
    wk.dense[2] = (double2 *)base;
    wk.dreal = (double *)(base + (((sizeof(double2) * (size_t)m * m) + 255) & ~(size_t)255));
    wk.dreal_elems = dense_real_elems(m);
    PARO_CHECK_LAUNCH(launch_heev(static_cast<hipStream_t>(s), wk, m, (const double2 *)A, w, (double2 *)V));
    return PARO_OK;
}

}  // extern "C"
