// Drivers of the hot path: H psi, the source problems (Algorithm 1, step 3),
// Rayleigh-Ritz (step 4), residuals and the ParO outer loop (steps 1, 3-5;
// Algorithm 2 for the MParO I variant).
#include <cmath>
#include <vector>

#include "paro_internal.h"

namespace paro {

static hipError_t apply_full(const Plan &pl, const Workspace &w, int nb, const double2 *x, int64_t ld, double2 *out,
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
static hipError_t source_solve(const Plan &pl, const Workspace &w, int nb, const double2 *psi, const double2 *hpsi,
                               int64_t ld, const double *eps, const double *shift, int ncg, double2 *u, int64_t ldu,
                               int32_t *band_flags, int mode = 0)
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

// H x in single precision (FP32 plan tables, FP32 matrix cores).
static hipError_t apply_full(const Plan &pl, const Workspace &w, int nb, const float2 *x, int64_t ld, float2 *out,
                             const double *shift)
{
    hipError_t e = launch_local_apply(pl, w, nb, x, ld, out, shift, nullptr, nullptr, false, nullptr, nullptr);
    if (e != hipSuccess || pl.nproj == 0) return e;
    float2 *P = reinterpret_cast<float2 *>(w.P);
    e = gemm_hn(pl.stream, pl.nproj, nb, pl.ng, pl.beta32, pl.ldv, x, ld, P, pl.nproj, w.part, w.part_elems, pl.dkb,
                nullptr);
    if (e != hipSuccess) return e;
    return gemm_nn(pl.stream, pl.ng, nb, pl.nproj, pl.beta32, pl.ldv, P, pl.nproj, out, ld, true);
}

// Mixed-precision source problems: the correction d = u - psi solves
// (H - sigma) d = eps psi - H psi (the same problem as source_solve, moved
// by the FP64 psi), by n_cg PCG steps from d = 0 with FP32 vectors, FP32
// applies of H and FP64 scalars; the right-hand side is formed in FP64 from
// the carried FP64 H psi, and u = psi + d (or u = d when correction) is
// written in FP64.  The FP64 Rayleigh-Ritz that follows acts as the
// refinement: the FP32 error is relative to d, which vanishes as the bands
// converge.
static hipError_t source_solve_mixed(const Plan &pl, const Workspace &w, int nb, const double2 *psi,
                                     const double2 *hpsi, int64_t ld, const double *eps, const double *shift, int ncg,
                                     double2 *u, int64_t ldu, int32_t *band_flags, bool correction)
{
    hipError_t e = launch_pcg_init_mixed(pl, w, nb, psi, hpsi, ld, eps, band_flags);
    double *pq_parts = w.dots + (size_t)DOT_PQ * nb * kMaxParts;
    float2 *P = reinterpret_cast<float2 *>(w.P);
    for (int k = 1; k <= ncg && e == hipSuccess; ++k) {
        int npq = 0;
        e = launch_local_apply(pl, w, nb, w.z32, pl.ldv, w.q32, shift, w.p32, w.sc + SC_BETA * nb, k == 1, pq_parts,
                               &npq);
        if (e == hipSuccess && pl.nproj > 0) {
            e = gemm_hn(pl.stream, pl.nproj, nb, pl.ng, pl.beta32, pl.ldv, w.p32, pl.ldv, P, pl.nproj, w.part,
                        w.part_elems, pl.dkb, w.sc + SC_NLQ * nb);
            if (e == hipSuccess)
                e = gemm_nn(pl.stream, pl.ng, nb, pl.nproj, pl.beta32, pl.ldv, P, pl.nproj, w.q32, pl.ldv, true);
        }
        if (e == hipSuccess) e = launch_pcg_update_mixed(pl, w, nb, npq, band_flags);
    }
    if (e == hipSuccess) e = launch_finish_correction(pl, w, nb, correction ? nullptr : psi, ld, u, ldu);
    return e;
}

static hipError_t rayleigh_ritz(const Plan &pl, const Workspace &w, int m, int nkeep, const double2 *U,
                                const double2 *W, int64_t ld, double *eps, double2 *psi, double2 *hpsi, int64_t ldo)
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

int32_t paro_apply_h_f32(paro_plan plan, int32_t nb, const float *psi, int64_t ld, const double *shift, float *hpsi,
                         void *ws, size_t ws_bytes)
{
    if (!plan || nb <= 0 || !psi || !hpsi) {
        set_error("paro_apply_h_f32: bad argument");
        return PARO_EINVAL;
    }
    const Plan &pl = plan->pl;
    if (ld < pl.ng) {
        set_error("paro_apply_h_f32: ld < n_g");
        return PARO_EINVAL;
    }
    const int nbw = (nb + 1) / 2;
    int32_t rc = check_ws(pl, nbw, ws, ws_bytes);
    if (rc) return rc;
    Workspace w = carve_workspace(pl, nbw, ws);
    PARO_CHECK_LAUNCH(apply_full(pl, w, nb, (const float2 *)psi, ld, (float2 *)hpsi, shift));
    return PARO_OK;
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
                                         n_cg, (double2 *)u, ld, band_flags, false));
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

int32_t paro_iterate(paro_plan plan, int32_t nb, double *psi_, double *hpsi_, int64_t ld, double *eps, double *sigma,
                     const paro_iter_opts *opts, double *stats, void *ws, size_t ws_bytes, int32_t *n_done)
{
    if (!plan || nb <= 0 || !psi_ || !hpsi_ || !eps || !sigma || !opts || opts->n_outer < 0 || opts->n_cg < 0 ||
        nb > 512 ||
        (opts->variant != PARO_VARIANT_PARO && opts->variant != PARO_VARIANT_MPARO1 &&
         opts->variant != PARO_VARIANT_MPARO2) ||
        (opts->shift_mode != PARO_SHIFT_FIXED && opts->shift_mode != PARO_SHIFT_ADAPTIVE) ||
        (opts->precision != PARO_PREC_FP64 && opts->precision != PARO_PREC_MIXED)) {
        set_error("paro_iterate: bad argument");
        return PARO_EINVAL;
    }
    const Plan &pl = plan->pl;
    if (ld < pl.ng) {
        set_error("paro_iterate: ld < n_g");
        return PARO_EINVAL;
    }
    if (opts->variant == PARO_VARIANT_MPARO2 && opts->precision != PARO_PREC_FP64) {
        set_error("paro_iterate: MParO II runs in FP64 only");
        return PARO_EUNSUP;
    }
    int32_t rc = check_ws(pl, nb, ws, ws_bytes);
    if (rc) return rc;
    Workspace w = carve_workspace(pl, nb, ws);
    double2 *psi = (double2 *)psi_, *hpsi = (double2 *)hpsi_;
    const int64_t lv = pl.ldv;
    hipStream_t st = pl.stream;
    const int row = 2 * nb + 2;
    int32_t *conv = reinterpret_cast<int32_t *>(w.scal + 1);
    if (n_done) *n_done = 0;
    if (opts->initial_rr) {
        PARO_CHECK_LAUNCH(launch_copy_bands(st, nb, pl.ng, psi, ld, w.U, lv));
        PARO_CHECK_LAUNCH(apply_full(pl, w, nb, w.U, lv, w.W, nullptr));
        PARO_CHECK_LAUNCH(rayleigh_ritz(pl, w, nb, nb, w.U, w.W, lv, eps, psi, hpsi, ld));
    }
    PARO_CHECK_LAUNCH(launch_residuals(pl, w, nb, psi, hpsi, ld, eps, w.res));
    PARO_CHECK_LAUNCH(launch_bookkeeping(pl, nb, *opts, eps, w.res, w.sig_all, sigma, stats, conv));
    std::vector<int32_t> hflags(nb);
    for (int it = 0; it < opts->n_outer; ++it) {
        if (opts->tol_res > 0.0) {
            int32_t c = 0;
            PARO_HIP_TRY(hipMemcpyAsync(&c, conv, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            PARO_HIP_TRY(hipStreamSynchronize(st));
            if (c) break;
        }
        const bool mparo = opts->variant != PARO_VARIANT_PARO;
        double2 *Ut = mparo ? w.U + (size_t)nb * lv : w.U;  // u (Algorithm 1) or e (Algorithms 2, 3)
        for (int attempt = 0; attempt < 2; ++attempt) {
            if (opts->precision == PARO_PREC_MIXED)
                PARO_CHECK_LAUNCH(source_solve_mixed(pl, w, nb, psi, hpsi, ld, eps, w.sig_all, opts->n_cg, Ut, lv,
                                                     w.iflags + nb, mparo));
            else
                PARO_CHECK_LAUNCH(source_solve(pl, w, nb, psi, hpsi, ld, eps, w.sig_all, opts->n_cg, Ut, lv,
                                               w.iflags + nb, opts->variant));
            if (opts->shift_mode != PARO_SHIFT_ADAPTIVE) break;
            // on negative curvature redo the source problems with sigma_lb
            double scur = 0.0;
            PARO_HIP_TRY(hipMemcpyAsync(hflags.data(), w.iflags + nb, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, st));
            PARO_HIP_TRY(hipMemcpyAsync(&scur, sigma, sizeof(double), hipMemcpyDeviceToHost, st));
            PARO_HIP_TRY(hipStreamSynchronize(st));
            bool neg = false;
            for (int b = 0; b < nb; ++b) neg = neg || (hflags[b] & PARO_F_NEGCURV);
            if (!neg || scur == opts->sigma_lb || attempt == 1) break;
            paro_iter_opts fixed = *opts;
            fixed.shift_mode = PARO_SHIFT_FIXED;
            fixed.tol_res = 0.0;
            PARO_CHECK_LAUNCH(launch_bookkeeping(pl, nb, fixed, eps, w.res, w.sig_all, sigma, nullptr, conv));
        }
        if (mparo) {
            // span{psi, e/|e|}, e from the correction equation (Algorithms 2, 3)
            PARO_CHECK_LAUNCH(launch_normalize_bands(pl, w, nb, Ut, lv));
            PARO_CHECK_LAUNCH(launch_copy_bands(st, nb, pl.ng, psi, ld, w.U, lv));
            PARO_CHECK_LAUNCH(launch_copy_bands(st, nb, pl.ng, hpsi, ld, w.W, lv));
            PARO_CHECK_LAUNCH(apply_full(pl, w, nb, Ut, lv, w.W + (size_t)nb * lv, nullptr));
            PARO_CHECK_LAUNCH(rayleigh_ritz(pl, w, 2 * nb, nb, w.U, w.W, lv, eps, psi, hpsi, ld));
        } else {
            PARO_CHECK_LAUNCH(apply_full(pl, w, nb, w.U, lv, w.W, nullptr));
            PARO_CHECK_LAUNCH(rayleigh_ritz(pl, w, nb, nb, w.U, w.W, lv, eps, psi, hpsi, ld));
        }
        PARO_CHECK_LAUNCH(launch_residuals(pl, w, nb, psi, hpsi, ld, eps, w.res));
        PARO_CHECK_LAUNCH(launch_bookkeeping(pl, nb, *opts, eps, w.res, w.sig_all, sigma,
                                             stats ? stats + (size_t)(it + 1) * row : nullptr, conv));
        if (n_done) *n_done = it + 1;
    }
    return PARO_OK;
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
