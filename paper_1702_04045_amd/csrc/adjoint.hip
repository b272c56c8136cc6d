// Reverse-mode derivative of the band energy after K truncated outer
// iterations of Algorithm 1 (Section 3) at a fixed shift, with respect to
// the local potential on the FFT grid and the KB projector centres.
//
// The map differentiated is the one paro_iterate computes with the fixed
// shift sigma and no tolerance, from a trial block Psi_T:
//   (eps^0, psi^0, Hpsi^0) = RR(Psi_T, H Psi_T)                     (step 1)
//   for n = 1..K: u_b = PCG_b(psi_b^{n-1}, Hpsi_b^{n-1}, eps_b^{n-1})  (step 3)
//                 (eps^n, psi^n, Hpsi^n) = RR(U, H U)                 (step 4)
//   E = sum_b w_b eps_b^K.
// Forward pass: the K + 1 Rayleigh-Ritz outputs are kept (one checkpoint
// per outer iteration).  Backward pass, n = K..1: the outer iteration is
// recomputed from checkpoint n - 1 with every PCG iterate kept (p_k, q_k =
// (H - sigma) p_k, r_{k+1}, z_{k+1} and the scalars), then
//   - Rayleigh-Ritz backward: with H_s C = S C Lambda, C^H S C = I and
//     Gb = C^H Cbar, the adjoints of H_s = U^H W and S = U^H U are
//     Abar = herm(C Pa C^H), Pa = diag(lambda_bar) + Gb o F,
//     Bbar = -herm(C Pb C^H), Pb_ii = lambda_bar_i lambda_i + Re Gb_ii / 2,
//     Pb_ij = Gb_ij F_ij lambda_j, F_ij = 1 / (lambda_j - lambda_i) (i != j);
//     Ubar = Psibar C^H + W Abar + 2 U Bbar, Wbar = Hpsibar C^H + U Abar;
//   - W = H U: Ubar += H Wbar;
//   - PCG backward, step by step in reverse: the adjoints of alpha, beta,
//     gamma, p^H q and of the Teter scale tau from dot products, then
//     rbar, qbar = -alpha rbar + pibar p, pbar = beta pbar' + alpha ubar +
//     pibar q + (H - sigma) qbar, down to psibar, Hpsibar and epsbar of the
//     previous Rayleigh-Ritz outputs.
// Every application of H to a vector x whose adjoint is y contributes
// Re <y, dH x> to the gradient: for V_j the grid value
// (1/N) Re(conj(y(r_j)) x(r_j)) and for R_p the derivative of the nonlocal
// form Re sum_p d_p conj(beta_p^H y) (beta_p^H x).  Both are bilinear, so
// they are formed from the quadratic forms of the density (paro_density)
// and the projector gradient (paro_projector_gradient) by polarisation:
// Re(conj(y) x) = (|y + x|^2 - |y - x|^2) / 4, on the 2 nb vectors y +- x
// with weights +-1/4.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fft_device.h"
#include "paro_internal.h"
#include "reduce_device.h"

namespace paro {

namespace {

constexpr int kAdjThreads = 256;
constexpr int kAdjChunk = 2048;  // sphere points per work-group
enum { AD_1 = 0, AD_2, AD_3, AD_4, AD_5, AD_6, AD_7, kAdjDots };
// per-band scalars of one traced PCG step: gamma_k, p^H q, beta_{k-1}, updated (1/0)
constexpr int kStepScal = 4;

inline unsigned nchunks(int64_t ng) { return (unsigned)((ng + kAdjChunk - 1) / kAdjChunk); }

__device__ __forceinline__ double teter_k(double x)
{
    const double num = 27.0 + 18.0 * x + 12.0 * x * x + 8.0 * x * x * x;
    return num / (num + 16.0 * x * x * x * x);
}
// dK/dx of the Teter ratio
__device__ __forceinline__ double teter_dk(double x)
{
    const double num = 27.0 + 18.0 * x + 12.0 * x * x + 8.0 * x * x * x;
    const double dnum = 18.0 + 24.0 * x + 24.0 * x * x;
    const double den = num + 16.0 * x * x * x * x;
    const double dden = dnum + 64.0 * x * x * x;
    return (dnum * den - num * dden) / (den * den);
}
__device__ __forceinline__ double re_dot(double2 a, double2 b) { return a.x * b.x + a.y * b.y; }

__device__ __forceinline__ double sum_parts(const double *p, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += p[i];
    return s;
}

__global__ void k_fill_f64(int n, double *__restrict__ p, double v)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_c128(int64_t n, double2 *__restrict__ p)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_double2(0.0, 0.0);
}

// After the apply of PCG step k (before the update): gamma_k, p_k^H q_k
// (local parts plus the nonlocal quadratic form), beta_{k-1} (the one p_k was
// formed with) and whether the update runs (active, p^H q > 0); tau once.
// A band that stopped (negative curvature, or its residual fell below the
// relative limit) has no update at the later steps: the backward pass
// takes those steps as the identity, the derivative along that branch.
__global__ void k_trace_scalars(int nb, int npq, const double *__restrict__ dots_pq, const double *__restrict__ sc,
                                const int32_t *__restrict__ active, double *__restrict__ out,
                                double *__restrict__ tau_out)
{
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const double pq = sum_parts(dots_pq + (size_t)b * kMaxParts, npq) + sc[SC_NLQ * nb + b];
        const bool upd = active[b] && pq > 0.0;
        out[kStepScal * b + 0] = sc[SC_GAMMA * nb + b];
        out[kStepScal * b + 1] = pq;
        out[kStepScal * b + 2] = sc[SC_BETA * nb + b];
        out[kStepScal * b + 3] = upd ? 1.0 : 0.0;
        if (tau_out) tau_out[b] = sc[SC_TAU * nb + b];
    }
}

// Partial dot products of the reverse of PCG step k (primes: index k + 1):
// D1 = Re<pbar', p>, D2 = Re<rbar, q>, D3 = Re<K pbar', q>, D4 = Re<z', q>,
// D5 = Re<ubar, p>, D6 = sum dK/dtau Re(conj(pbar') r'), D7 = sum dK/dtau |r'|^2.
__global__ void __launch_bounds__(kAdjThreads)
k_adj_dots(int64_t ng, int nb, int64_t ldv, int last, const double *__restrict__ st_k, const double *__restrict__ st_n,
           const double2 *__restrict__ pbn, const double2 *__restrict__ p, const double2 *__restrict__ q,
           const double2 *__restrict__ rn, const double2 *__restrict__ zn, const double2 *__restrict__ rb,
           const double2 *__restrict__ ub, const double *__restrict__ kin, const double *__restrict__ tau_b,
           double *__restrict__ dots)
{
    __shared__ double red[kAdjThreads / 64];
    const int band = blockIdx.y;
    const double tau = tau_b[band];
    const bool act = st_k[kStepScal * band + 3] > 0.5;
    const int has_next = act && !last && st_n[kStepScal * band + 3] > 0.5;
    const size_t o = (size_t)band * ldv;
    double d[kAdjDots] = {0, 0, 0, 0, 0, 0, 0};
    const int64_t g0 = (int64_t)blockIdx.x * kAdjChunk;
    const int64_t g1 = g0 + kAdjChunk < ng ? g0 + kAdjChunk : ng;
    for (int64_t g = g0 + threadIdx.x; g < g1 && act; g += kAdjThreads) {
        const double2 pv = p[o + g], qv = q[o + g], rv = rn[o + g], zv = zn[o + g], rbv = rb[o + g], uv = ub[o + g];
        const double x = kin[g] / tau;
        const double dkt = teter_dk(x) * (-kin[g] / (tau * tau));
        d[AD_2] += re_dot(rbv, qv);
        d[AD_4] += re_dot(zv, qv);
        d[AD_5] += re_dot(uv, pv);
        d[AD_7] += dkt * re_dot(rv, rv);
        if (has_next) {
            const double2 pn = pbn[o + g];
            const double k = teter_k(x);
            d[AD_1] += re_dot(pn, pv);
            d[AD_3] += k * re_dot(pn, qv);
            d[AD_6] += dkt * re_dot(pn, rv);
        }
    }
#pragma unroll
    for (int i = 0; i < kAdjDots; ++i) {
        const double v = block_sum<kAdjThreads>(d[i], red);
        if (threadIdx.x == 0) dots[((size_t)i * nb + band) * kMaxParts + blockIdx.x] = v;
    }
}

// Scalar adjoints of PCG step k.  gbar: in gamma-bar_{k+1} accumulated so
// far, out gamma-bar_k; taub: accumulated tau-bar.  coef per band: 2
// gamma-bar_{k+1}, alpha_k, pi-bar_k, beta_k.
__global__ void k_adj_scalars(int nb, int nparts, int last, const double *__restrict__ dots,
                              const double *__restrict__ st_k, const double *__restrict__ st_n,
                              double *__restrict__ gbar, double *__restrict__ taub, double *__restrict__ coef)
{
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        auto D = [&](int i) { return sum_parts(dots + ((size_t)i * nb + b) * kMaxParts, nparts); };
        if (!(st_k[kStepScal * b + 3] > 0.5)) {
            // no update at this step (the band had stopped): the step is the identity
            coef[4 * b + 0] = coef[4 * b + 1] = coef[4 * b + 2] = coef[4 * b + 3] = 0.0;
            continue;
        }
        const bool has_next = !last && st_n[kStepScal * b + 3] > 0.5;
        const double g = st_k[kStepScal * b], pq = st_k[kStepScal * b + 1];
        const double alpha = g / pq;
        double beta = 0.0, gn = gbar[b], gk = 0.0;
        if (has_next) {
            beta = st_n[kStepScal * b + 2];          // beta_k formed p_{k+1}
            const double gnext = st_n[kStepScal * b];  // gamma_{k+1}
            const double bbar = D(AD_1);
            gn += bbar / g;
            gk = -bbar * gnext / (g * g);
        }
        taub[b] += D(AD_6) + gn * D(AD_7);
        const double cz = 2.0 * gn;
        const double abar = -(D(AD_2) + D(AD_3) + cz * D(AD_4)) + D(AD_5);
        gk += abar / pq;
        const double pibar = -abar * g / (pq * pq);
        gbar[b] = gk;
        coef[4 * b + 0] = cz;
        coef[4 * b + 1] = alpha;
        coef[4 * b + 2] = pibar;
        coef[4 * b + 3] = beta;
    }
}

// rbar += K pbar' + 2 gbar' z'; qbar = -alpha rbar + pibar p;
// pbar = beta pbar' + alpha ubar + pibar q; s+- = qbar +- p (polarisation pair).
__global__ void __launch_bounds__(kAdjThreads)
k_adj_vec(int64_t ng, int nb, int64_t ldv, int last, const double *__restrict__ st_k, const double *__restrict__ st_n,
          const double *__restrict__ coef, const double2 *__restrict__ pbn, const double2 *__restrict__ p,
          const double2 *__restrict__ q,
          const double2 *__restrict__ zn, const double2 *__restrict__ ub, const double *__restrict__ kin,
          const double *__restrict__ tau_b, double2 *__restrict__ rb, double2 *__restrict__ qb,
          double2 *__restrict__ pb, double2 *__restrict__ spm)
{
    const int band = blockIdx.y;
    const double cz = coef[4 * band], alpha = coef[4 * band + 1], pibar = coef[4 * band + 2];
    const double beta = coef[4 * band + 3], tau = tau_b[band];
    const int has_next = !last && st_k[kStepScal * band + 3] > 0.5 && st_n[kStepScal * band + 3] > 0.5;
    const size_t o = (size_t)band * ldv, om = (size_t)(band + nb) * ldv;
    const int64_t g0 = (int64_t)blockIdx.x * kAdjChunk;
    const int64_t g1 = g0 + kAdjChunk < ng ? g0 + kAdjChunk : ng;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kAdjThreads) {
        const double2 pv = p[o + g], qv = q[o + g], zv = zn[o + g], uv = ub[o + g];
        double2 r = rb[o + g];
        double2 pn = make_double2(0.0, 0.0);
        if (has_next) {
            pn = pbn[o + g];
            const double k = teter_k(kin[g] / tau);
            r.x += k * pn.x;
            r.y += k * pn.y;
        }
        r.x += cz * zv.x;
        r.y += cz * zv.y;
        rb[o + g] = r;
        const double2 qbv = make_double2(-alpha * r.x + pibar * pv.x, -alpha * r.y + pibar * pv.y);
        qb[o + g] = qbv;
        pb[o + g] = make_double2(beta * pn.x + alpha * uv.x + pibar * qv.x, beta * pn.y + alpha * uv.y + pibar * qv.y);
        spm[o + g] = make_double2(qbv.x + pv.x, qbv.y + pv.y);
        spm[om + g] = make_double2(qbv.x - pv.x, qbv.y - pv.y);
    }
}

// y += x (nb bands, ldv)
__global__ void __launch_bounds__(kAdjThreads)
k_axpy_bands(int64_t ng, int64_t ldv, const double2 *__restrict__ x, double2 *__restrict__ y)
{
    const size_t o = (size_t)blockIdx.y * ldv;
    const int64_t g0 = (int64_t)blockIdx.x * kAdjChunk;
    const int64_t g1 = g0 + kAdjChunk < ng ? g0 + kAdjChunk : ng;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kAdjThreads) {
        const double2 a = x[o + g], b = y[o + g];
        y[o + g] = make_double2(a.x + b.x, a.y + b.y);
    }
}

// s+- = a +- b (nb bands each, a with leading dimension lda, b with ldb)
__global__ void __launch_bounds__(kAdjThreads)
k_polar_pair(int64_t ng, int nb, const double2 *__restrict__ a, int64_t lda, const double2 *__restrict__ b,
             int64_t ldb, double2 *__restrict__ spm, int64_t ldv)
{
    const int band = blockIdx.y;
    const int64_t g0 = (int64_t)blockIdx.x * kAdjChunk;
    const int64_t g1 = g0 + kAdjChunk < ng ? g0 + kAdjChunk : ng;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kAdjThreads) {
        const double2 x = a[band * lda + g], y = b[band * ldb + g];
        spm[(size_t)band * ldv + g] = make_double2(x.x + y.x, x.y + y.y);
        spm[(size_t)(band + nb) * ldv + g] = make_double2(x.x - y.x, x.y - y.y);
    }
}

// Partial sums of the PCG start (k = 0 reversed; p_0 = z_0 = K r_0,
// r_0 = eps psi - Hpsi, u_0 = psi, tau = <psi|T|psi>/<psi|psi>):
// D1 = sum dK/dtau Re(conj(pbar_0) r_0), D2 = sum dK/dtau |r_0|^2, D3 = Re<rbar, psi>,
// D4 = Re<K pbar_0, psi>, D5 = Re<z_0, psi>, D6 = |psi|^2.
__global__ void __launch_bounds__(kAdjThreads)
k_adj0_dots(int64_t ng, int nb, int64_t ldv, const double2 *__restrict__ pb, const double2 *__restrict__ r0,
            const double2 *__restrict__ z0, const double2 *__restrict__ rb, const double2 *__restrict__ psi,
            int64_t ld, const double *__restrict__ kin, const double *__restrict__ tau_b, double *__restrict__ dots)
{
    __shared__ double red[kAdjThreads / 64];
    const int band = blockIdx.y;
    const double tau = tau_b[band];
    const size_t o = (size_t)band * ldv;
    double d[kAdjDots] = {0, 0, 0, 0, 0, 0, 0};
    const int64_t g0 = (int64_t)blockIdx.x * kAdjChunk;
    const int64_t g1 = g0 + kAdjChunk < ng ? g0 + kAdjChunk : ng;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kAdjThreads) {
        const double2 pv = pb[o + g], rv = r0[o + g], zv = z0[o + g], rbv = rb[o + g], xv = psi[band * ld + g];
        const double x = kin[g] / tau;
        const double dkt = teter_dk(x) * (-kin[g] / (tau * tau));
        d[AD_1] += dkt * re_dot(pv, rv);
        d[AD_2] += dkt * re_dot(rv, rv);
        d[AD_3] += re_dot(rbv, xv);
        d[AD_4] += teter_k(x) * re_dot(pv, xv);
        d[AD_5] += re_dot(zv, xv);
        d[AD_6] += re_dot(xv, xv);
    }
#pragma unroll
    for (int i = 0; i < kAdjDots; ++i) {
        const double v = block_sum<kAdjThreads>(d[i], red);
        if (threadIdx.x == 0) dots[((size_t)i * nb + band) * kMaxParts + blockIdx.x] = v;
    }
}

// coef0 per band: 2 gbar_0, eps, 2 taubar / |psi|^2, tau; epsbar = Re<rbar_0, psi>.
__global__ void k_adj0_scalars(int nb, int nparts, const double *__restrict__ dots, const double *__restrict__ gbar,
                               const double *__restrict__ taub, const double *__restrict__ eps,
                               const double *__restrict__ tau_b, double *__restrict__ coef, double *__restrict__ epsbar)
{
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        auto D = [&](int i) { return sum_parts(dots + ((size_t)i * nb + b) * kMaxParts, nparts); };
        const double g0 = gbar[b];
        const double tb = taub[b] + D(AD_1) + g0 * D(AD_2);
        epsbar[b] = D(AD_3) + D(AD_4) + 2.0 * g0 * D(AD_5);
        coef[4 * b + 0] = 2.0 * g0;
        coef[4 * b + 1] = eps[b];
        coef[4 * b + 2] = 2.0 * tb / D(AD_6);
        coef[4 * b + 3] = tau_b[b];
    }
}

// rbar_0 = rbar + K pbar_0 + 2 gbar_0 z_0; psibar = eps rbar_0 + ubar + (2 taubar/|psi|^2)(kin - tau) psi;
// Hpsibar = -rbar_0.
__global__ void __launch_bounds__(kAdjThreads)
k_adj0_vec(int64_t ng, int64_t ldv, const double *__restrict__ coef, const double2 *__restrict__ pb,
           const double2 *__restrict__ z0, const double2 *__restrict__ rb, const double2 *__restrict__ ub,
           const double2 *__restrict__ psi, int64_t ld, const double *__restrict__ kin, double2 *__restrict__ psibar,
           double2 *__restrict__ hbar)
{
    const int band = blockIdx.y;
    const double c2g = coef[4 * band], e = coef[4 * band + 1], ct = coef[4 * band + 2], tau = coef[4 * band + 3];
    const size_t o = (size_t)band * ldv;
    const int64_t g0 = (int64_t)blockIdx.x * kAdjChunk;
    const int64_t g1 = g0 + kAdjChunk < ng ? g0 + kAdjChunk : ng;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kAdjThreads) {
        const double2 pv = pb[o + g], zv = z0[o + g], rbv = rb[o + g], uv = ub[o + g], xv = psi[band * ld + g];
        const double k = teter_k(kin[g] / tau);
        const double2 r0b = make_double2(rbv.x + k * pv.x + c2g * zv.x, rbv.y + k * pv.y + c2g * zv.y);
        const double s = ct * (kin[g] - tau);
        psibar[o + g] = make_double2(e * r0b.x + uv.x + s * xv.x, e * r0b.y + uv.y + s * xv.y);
        hbar[o + g] = make_double2(-r0b.x, -r0b.y);
    }
}

// Small dense products for the Rayleigh-Ritz adjoint (m <= 1024, column-major):
// C = op(A) op(B), op = identity or conjugate transpose (ha, hb).
constexpr int kSmallTile = 16;
__global__ void __launch_bounds__(kSmallTile * kSmallTile)
k_small_gemm(int m, const double2 *__restrict__ A, int ha, const double2 *__restrict__ B, int hb,
             double2 *__restrict__ C)
{
    __shared__ double2 ta[kSmallTile][kSmallTile + 1], tb[kSmallTile][kSmallTile + 1];
    const int tx = threadIdx.x % kSmallTile, ty = threadIdx.x / kSmallTile;
    const int i = blockIdx.x * kSmallTile + tx, j = blockIdx.y * kSmallTile + ty;
    double2 acc = make_double2(0.0, 0.0);
    for (int k0 = 0; k0 < m; k0 += kSmallTile) {
        // ta[ty][tx] = op(A)(i, k0 + ty); tb[ty][tx] = op(B)(k0 + tx, j)
        {
            const int r = i, c = k0 + ty;
            double2 a = make_double2(0.0, 0.0);
            if (r < m && c < m) a = ha ? make_double2(A[(size_t)r * m + c].x, -A[(size_t)r * m + c].y) : A[(size_t)c * m + r];
            ta[ty][tx] = a;
        }
        {
            const int r = k0 + tx, c = j;
            double2 b = make_double2(0.0, 0.0);
            if (r < m && c < m) b = hb ? make_double2(B[(size_t)r * m + c].x, -B[(size_t)r * m + c].y) : B[(size_t)c * m + r];
            tb[ty][tx] = b;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kSmallTile; ++kk) {
            const double2 a = ta[kk][tx], b = tb[ty][kk];
            acc.x += a.x * b.x - a.y * b.y;
            acc.y += a.x * b.y + a.y * b.x;
        }
        __syncthreads();
    }
    if (i < m && j < m) C[(size_t)j * m + i] = acc;
}

// out = s (X + X^H) / 2
__global__ void k_herm_scale(int m, const double2 *__restrict__ X, double s, double2 *__restrict__ out)
{
    const int64_t mm = (int64_t)m * m;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < mm; q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q % m), j = (int)(q / m);
        const double2 a = X[q], b = X[(size_t)i * m + j];
        out[q] = make_double2(0.5 * s * (a.x + b.x), 0.5 * s * (a.y - b.y));
    }
}

// Pa_ij = i == j ? lambda_bar_i : G_ij / (lambda_j - lambda_i)
// Pb_ij = i == j ? lambda_bar_i lambda_i + Re G_ii / 2 : G_ij lambda_j / (lambda_j - lambda_i)
__global__ void k_rr_adj_mid(int m, const double *__restrict__ lam, const double *__restrict__ lbar,
                             const double2 *__restrict__ G, double2 *__restrict__ Pa, double2 *__restrict__ Pb)
{
    const int64_t mm = (int64_t)m * m;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < mm; q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q % m), j = (int)(q / m);
        const double2 g = G[q];
        if (i == j) {
            Pa[q] = make_double2(lbar[i], 0.0);
            Pb[q] = make_double2(lbar[i] * lam[i] + 0.5 * g.x, 0.0);
        } else {
            const double f = 1.0 / (lam[j] - lam[i]);
            Pa[q] = make_double2(g.x * f, g.y * f);
            Pb[q] = make_double2(g.x * f * lam[j], g.y * f * lam[j]);
        }
    }
}

// out = A^H (m x m)
__global__ void k_conj_transpose(int m, const double2 *__restrict__ A, double2 *__restrict__ out)
{
    const int64_t mm = (int64_t)m * m;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < mm; q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q % m), j = (int)(q / m);
        const double2 a = A[(size_t)i * m + j];
        out[q] = make_double2(a.x, -a.y);
    }
}

// C += D (m x m)
__global__ void k_add_small(int64_t n, const double2 *__restrict__ D, double2 *__restrict__ C)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        C[q] = make_double2(C[q].x + D[q].x, C[q].y + D[q].y);
}

// y += x (n doubles)
__global__ void k_add_f64(int n, const double *__restrict__ x, double *__restrict__ y)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) y[i] += x[i];
}

// E = sum_b w_b eps_b
__global__ void k_weighted_sum(int nb, const double *__restrict__ w, const double *__restrict__ eps,
                               double *__restrict__ out)
{
    __shared__ double red[4];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += w[b] * eps[b];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ void k_scale_f64(int64_t n, double s, double *__restrict__ p)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] *= s;
}

}  // namespace

// ---------------------------------------------------------------- host side

// Carve-up of the adjoint workspace: the solver workspace for nb bands,
// then checkpoints, the PCG trace and the adjoint vectors.
struct AdjWs {
    Workspace w;
    double2 *ck_psi, *ck_h;   // (K + 1) x nb x ldv
    double *ck_eps;           // (K + 1) x nb
    double2 *tr_p, *tr_q;     // n_cg x nb x ldv
    double2 *tr_r, *tr_z;     // (n_cg + 1) x nb x ldv: r_0 .. r_ncg, z_0 .. z_ncg
    double *tr_sc;            // n_cg x nb x kStepScal
    double *tau;              // nb
    double2 *ub, *wb, *rb, *pb, *pbn, *qb, *tmp, *psib, *hb;  // nb x ldv each
    double2 *psi_t, *h_t;     // nb x ldv: recomputed outputs (discarded)
    double2 *spm;             // 2 nb x ldv: polarisation pairs
    double *eps_t, *epsb, *gbar, *taub, *coef, *pol_w, *adots;  // small
    double2 *sm[8];           // m x m: Cbar, Cbar2, CH, G, Pa, Pb, X, Y
    double2 *dens_sticks;     // density workspace
    double *dens_part;
    ProjGradWs pg;
    double *dd_t, *dR_t;      // n_proj, 3 n_proj
};

static size_t adj_layout(const Plan &pl, int nb, int K, int ncg, void *ws, AdjWs *a)
{
    const size_t ldv = pl.ldv, vb = sizeof(double2) * nb * ldv;
    char *base = static_cast<char *>(ws);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off = (off + bytes + 255) & ~(size_t)255;
        return p;
    };
    const size_t wsb = workspace_bytes(pl, nb);
    char *wbase = take(wsb);
    AdjWs A{};
    if (base) A.w = carve_workspace(pl, nb, wbase);
    A.ck_psi = (double2 *)take(vb * (K + 1));
    A.ck_h = (double2 *)take(vb * (K + 1));
    A.ck_eps = (double *)take(sizeof(double) * nb * (K + 1));
    A.tr_p = (double2 *)take(vb * ncg);
    A.tr_q = (double2 *)take(vb * ncg);
    A.tr_r = (double2 *)take(vb * (ncg + 1));
    A.tr_z = (double2 *)take(vb * (ncg + 1));
    A.tr_sc = (double *)take(sizeof(double) * kStepScal * nb * (ncg + 1));
    A.tau = (double *)take(sizeof(double) * nb);
    double2 **vecs[] = {&A.ub, &A.wb, &A.rb, &A.pb, &A.pbn, &A.qb, &A.tmp, &A.psib, &A.hb, &A.psi_t, &A.h_t};
    for (double2 **v : vecs) *v = (double2 *)take(vb);
    A.spm = (double2 *)take(2 * vb);
    double **sm[] = {&A.eps_t, &A.epsb, &A.gbar, &A.taub, &A.coef, &A.pol_w};
    for (double **v : sm) *v = (double *)take(sizeof(double) * 4 * 2 * nb);
    A.adots = (double *)take(sizeof(double) * kAdjDots * nb * kMaxParts);
    for (int i = 0; i < 8; ++i) A.sm[i] = (double2 *)take(sizeof(double2) * (size_t)nb * nb);
    size_t part_off = 0;
    const size_t db = density_workspace_bytes(pl, 2 * nb, &part_off);
    char *dbase = take(db);
    A.dens_sticks = (double2 *)dbase;
    A.dens_part = dbase ? (double *)(dbase + part_off) : nullptr;
    size_t pgb = 0;
    proj_grad_workspace(pl, 2 * nb, nullptr, &pgb);
    char *pgbase = take(pgb);
    if (base) A.pg = proj_grad_workspace(pl, 2 * nb, pgbase, nullptr);
    A.dd_t = (double *)take(sizeof(double) * std::max(1, pl.nproj));
    A.dR_t = (double *)take(sizeof(double) * 3 * std::max(1, pl.nproj));
    if (a) *a = A;
    return off;
}

namespace {

inline dim3 vgrid(const Plan &pl, int nb) { return dim3(nchunks(pl.ng), nb); }

// Re <y, dH x> for every band (y and x nb x ld blocks) into the gradient
// accumulators: density and projector gradient of the pairs y +- x with
// weights +-1/4 (rho is scaled by 1/N at the end).
hipError_t accumulate_cross(const Plan &pl, const AdjWs &a, int nb, const double2 *y, int64_t ldy, const double2 *x,
                            int64_t ldx, double *rho, double *dR)
{
    hipLaunchKernelGGL(k_polar_pair, vgrid(pl, nb), dim3(kAdjThreads), 0, pl.stream, pl.ng, nb, y, ldy, x, ldx, a.spm,
                       pl.ldv);
    hipError_t e = launch_density(pl, a.dens_sticks, a.dens_part, 2 * nb, a.spm, pl.ldv, a.pol_w, rho, true);
    if (e != hipSuccess || pl.nproj == 0) return e;
    e = launch_projector_gradient(pl, a.pg, 2 * nb, a.spm, pl.ldv, a.pol_w, a.dd_t, a.dR_t);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_add_f64, dim3(1), dim3(256), 0, pl.stream, 3 * pl.nproj, a.dR_t, dR);
    return hipGetLastError();
}

// The PCG of one outer iteration with every iterate kept (the same launches
// as source_solve, mode 0, plus copies of p, q, r, z and the step scalars).
hipError_t pcg_traced(const Plan &pl, const AdjWs &a, int nb, const double2 *psi, const double2 *hpsi,
                      const double *eps, int ncg, double2 *u)
{
    const Workspace &w = a.w;
    const int64_t ldv = pl.ldv;
    const size_t vstride = (size_t)nb * ldv;
    hipError_t e = launch_pcg_init(pl, w, nb, psi, hpsi, ldv, eps, u, ldv, nullptr, false, nullptr);
    if (e != hipSuccess) return e;
    if ((e = launch_copy_bands(pl.stream, nb, pl.ng, w.r, ldv, a.tr_r, ldv)) != hipSuccess) return e;
    if ((e = launch_copy_bands(pl.stream, nb, pl.ng, w.z, ldv, a.tr_z, ldv)) != hipSuccess) return e;
    double *pq_parts = w.dots + (size_t)DOT_PQ * nb * kMaxParts;
    for (int k = 1; k <= ncg && e == hipSuccess; ++k) {
        int npq = 0;
        e = launch_local_apply(pl, w, nb, w.z, ldv, w.q, w.sig_all, w.p, w.sc + SC_BETA * nb, k == 1, pq_parts, &npq);
        if (e == hipSuccess && pl.nproj > 0) {
            e = gemm_hn(pl.stream, pl.nproj, nb, pl.ng, pl.beta, ldv, w.p, ldv, w.P, pl.nproj, w.part, w.part_elems,
                        pl.dkb, w.sc + SC_NLQ * nb);
            if (e == hipSuccess)
                e = gemm_nn(pl.stream, pl.ng, nb, pl.nproj, pl.beta, ldv, w.P, pl.nproj, w.q, ldv, true);
        }
        if (e != hipSuccess) break;
        const int j = k - 1;
        hipLaunchKernelGGL(k_trace_scalars, dim3(1), dim3(256), 0, pl.stream, nb, npq, pq_parts, w.sc, w.iflags,
                           a.tr_sc + (size_t)j * kStepScal * nb, j == 0 ? a.tau : nullptr);
        if ((e = launch_copy_bands(pl.stream, nb, pl.ng, w.p, ldv, a.tr_p + j * vstride, ldv)) != hipSuccess) break;
        if ((e = launch_copy_bands(pl.stream, nb, pl.ng, w.q, ldv, a.tr_q + j * vstride, ldv)) != hipSuccess) break;
        if ((e = launch_pcg_update(pl, w, nb, u, ldv, npq, nullptr)) != hipSuccess) break;
        if ((e = launch_copy_bands(pl.stream, nb, pl.ng, w.r, ldv, a.tr_r + (size_t)k * vstride, ldv)) != hipSuccess)
            break;
        if ((e = launch_copy_bands(pl.stream, nb, pl.ng, w.z, ldv, a.tr_z + (size_t)k * vstride, ldv)) != hipSuccess)
            break;
    }
    return e == hipSuccess ? hipGetLastError() : e;
}

// Rayleigh-Ritz backward (m = nb, all pairs kept).  In: U, W (nb x ldv),
// C = w.dense[4] and lambda of the forward, psibar, hbar, epsbar.  Out: ub =
// Ubar, wb = Wbar.
hipError_t rr_backward(const Plan &pl, const AdjWs &a, int m, const double2 *U, const double2 *W,
                       const double *lam, const double2 *psibar, const double2 *hbar, const double *epsbar)
{
    const Workspace &w = a.w;
    const int64_t ldv = pl.ldv;
    const double2 *C = w.dense[4];
    double2 *Cb = a.sm[0], *Cb2 = a.sm[1], *CH = a.sm[2], *G = a.sm[3], *Pa = a.sm[4], *Pb = a.sm[5], *X = a.sm[6],
            *Y = a.sm[7];
    const size_t mm = (size_t)m * m;
    const dim3 sg((m + kSmallTile - 1) / kSmallTile, (m + kSmallTile - 1) / kSmallTile), st(kSmallTile * kSmallTile);
    const dim3 eg((unsigned)std::min<size_t>((mm + 255) / 256, 4096));
    // Cbar = U^H psibar + W^H hbar
    hipError_t e = gemm_hn(pl.stream, m, m, pl.ng, U, ldv, psibar, ldv, Cb, m, w.part, w.part_elems, nullptr, nullptr);
    if (e == hipSuccess)
        e = gemm_hn(pl.stream, m, m, pl.ng, W, ldv, hbar, ldv, Cb2, m, w.part, w.part_elems, nullptr, nullptr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_add_small, eg, dim3(256), 0, pl.stream, (int64_t)mm, Cb2, Cb);
    // G = C^H Cbar; Pa, Pb
    hipLaunchKernelGGL(k_small_gemm, sg, st, 0, pl.stream, m, C, 1, Cb, 0, G);
    hipLaunchKernelGGL(k_rr_adj_mid, eg, dim3(256), 0, pl.stream, m, lam, epsbar, G, Pa, Pb);
    // Abar = herm(C Pa C^H) -> Pa;  -2 herm(C Pb C^H) -> Pb
    hipLaunchKernelGGL(k_small_gemm, sg, st, 0, pl.stream, m, C, 0, Pa, 0, X);
    hipLaunchKernelGGL(k_small_gemm, sg, st, 0, pl.stream, m, X, 0, C, 1, Y);
    hipLaunchKernelGGL(k_herm_scale, eg, dim3(256), 0, pl.stream, m, Y, 1.0, Pa);
    hipLaunchKernelGGL(k_small_gemm, sg, st, 0, pl.stream, m, C, 0, Pb, 0, X);
    hipLaunchKernelGGL(k_small_gemm, sg, st, 0, pl.stream, m, X, 0, C, 1, Y);
    hipLaunchKernelGGL(k_herm_scale, eg, dim3(256), 0, pl.stream, m, Y, -2.0, Pb);
    // C^H for the products with the long blocks
    hipLaunchKernelGGL(k_conj_transpose, eg, dim3(256), 0, pl.stream, m, C, CH);
    // Ubar = psibar C^H + W Abar + U (-2 herm(C Pb C^H)); Wbar = hbar C^H + U Abar
    if ((e = gemm_nn(pl.stream, pl.ng, m, m, psibar, ldv, CH, m, a.ub, ldv, false)) != hipSuccess) return e;
    if ((e = gemm_nn(pl.stream, pl.ng, m, m, W, ldv, Pa, m, a.ub, ldv, true)) != hipSuccess) return e;
    if ((e = gemm_nn(pl.stream, pl.ng, m, m, U, ldv, Pb, m, a.ub, ldv, true)) != hipSuccess) return e;
    if ((e = gemm_nn(pl.stream, pl.ng, m, m, hbar, ldv, CH, m, a.wb, ldv, false)) != hipSuccess) return e;
    return gemm_nn(pl.stream, pl.ng, m, m, U, ldv, Pa, m, a.wb, ldv, true);
}

// The adjoint of the PCG of one outer iteration (trace in a), from ubar =
// a.ub to psibar, hbar, epsbar of its inputs (a.psib, a.hb, a.epsb), with
// the gradient contributions of its applies.
hipError_t pcg_backward(const Plan &pl, const AdjWs &a, int nb, int ncg, const double2 *psi, const double *eps,
                        double *rho, double *dR)
{
    const Workspace &w = a.w;
    const int64_t ldv = pl.ldv;
    const size_t vstride = (size_t)nb * ldv;
    const unsigned nc = nchunks(pl.ng);
    const dim3 vg = vgrid(pl, nb), sb(256);
    const int64_t nvec = (int64_t)nb * ldv;
    const unsigned fg = (unsigned)std::min<int64_t>((nvec + 255) / 256, 65535);
    hipLaunchKernelGGL(k_fill_c128, dim3(fg), dim3(256), 0, pl.stream, nvec, a.rb);
    hipLaunchKernelGGL(k_fill_f64, dim3(1), sb, 0, pl.stream, nb, a.gbar, 0.0);
    hipLaunchKernelGGL(k_fill_f64, dim3(1), sb, 0, pl.stream, nb, a.taub, 0.0);
    double2 *pb = a.pb, *pbn = a.pbn;
    hipError_t e = hipSuccess;
    for (int j = ncg - 1; j >= 0 && e == hipSuccess; --j) {
        // per band, step j has a successor when the next step updated too
        const int last = j == ncg - 1 ? 1 : 0;
        const double *stk = a.tr_sc + (size_t)j * kStepScal * nb, *stn = a.tr_sc + (size_t)(j + 1) * kStepScal * nb;
        const double2 *p = a.tr_p + j * vstride, *q = a.tr_q + j * vstride;
        const double2 *rn = a.tr_r + (j + 1) * vstride, *zn = a.tr_z + (j + 1) * vstride;
        hipLaunchKernelGGL(k_adj_dots, vg, dim3(kAdjThreads), 0, pl.stream, pl.ng, nb, ldv, last, stk, stn, pbn, p, q,
                           rn, zn, a.rb, a.ub, pl.kin, a.tau, a.adots);
        hipLaunchKernelGGL(k_adj_scalars, dim3(1), sb, 0, pl.stream, nb, (int)nc, last, a.adots, stk, stn, a.gbar,
                           a.taub, a.coef);
        hipLaunchKernelGGL(k_adj_vec, vg, dim3(kAdjThreads), 0, pl.stream, pl.ng, nb, ldv, last, stk, stn, a.coef, pbn,
                           p, q, zn, a.ub, pl.kin, a.tau, a.rb, a.qb, pb, a.spm);
        // pbar += (H - sigma) qbar
        if ((e = apply_full(pl, w, nb, a.qb, ldv, a.tmp, w.sig_all)) != hipSuccess) break;
        hipLaunchKernelGGL(k_axpy_bands, vg, dim3(kAdjThreads), 0, pl.stream, pl.ng, ldv, a.tmp, pb);
        // Re <qbar, dH p>
        if ((e = launch_density(pl, a.dens_sticks, a.dens_part, 2 * nb, a.spm, ldv, a.pol_w, rho, true)) !=
            hipSuccess)
            break;
        if (pl.nproj > 0) {
            if ((e = launch_projector_gradient(pl, a.pg, 2 * nb, a.spm, ldv, a.pol_w, a.dd_t, a.dR_t)) != hipSuccess)
                break;
            hipLaunchKernelGGL(k_add_f64, dim3(1), sb, 0, pl.stream, 3 * pl.nproj, a.dR_t, dR);
        }
        std::swap(pb, pbn);
    }
    if (e != hipSuccess) return e;
    // p_0 = z_0 = K r_0, r_0 = eps psi - Hpsi, u_0 = psi, tau(psi); pbn holds pbar_0
    hipLaunchKernelGGL(k_adj0_dots, vg, dim3(kAdjThreads), 0, pl.stream, pl.ng, nb, ldv, pbn, a.tr_r, a.tr_z, a.rb,
                       psi, ldv, pl.kin, a.tau, a.adots);
    hipLaunchKernelGGL(k_adj0_scalars, dim3(1), sb, 0, pl.stream, nb, (int)nc, a.adots, a.gbar, a.taub, eps, a.tau,
                       a.coef, a.epsb);
    hipLaunchKernelGGL(k_adj0_vec, vg, dim3(kAdjThreads), 0, pl.stream, pl.ng, ldv, a.coef, pbn, a.tr_z, a.rb, a.ub,
                       psi, ldv, pl.kin, a.psib, a.hb);
    return hipGetLastError();
}

int32_t truncated_gradient(const Plan &pl, int nb, const double2 *trial, int64_t ld, double sigma, int K, int ncg,
                           const double *weights, double *energy, double *rho, double *dR, void *ws)
{
    AdjWs a{};
    adj_layout(pl, nb, K, ncg, ws, &a);
    const Workspace &w = a.w;
    const int64_t ldv = pl.ldv;
    const size_t vstride = (size_t)nb * ldv;
    hipStream_t st = pl.stream;
    const dim3 sb(256);
    const int64_t nv = (int64_t)pl.grid[0] * pl.grid[1] * pl.grid[2];
    const int64_t nvec = (int64_t)nb * ldv;
    const unsigned fg = (unsigned)std::min<int64_t>((nvec + 255) / 256, 65535);
    hipLaunchKernelGGL(k_fill_f64, dim3(1), sb, 0, st, nb, w.sig_all, sigma);
    hipLaunchKernelGGL(k_fill_f64, dim3(1), sb, 0, st, nb, a.pol_w, 0.25);
    hipLaunchKernelGGL(k_fill_f64, dim3(1), sb, 0, st, nb, a.pol_w + nb, -0.25);
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)std::min<int64_t>((nv + 255) / 256, 65535)), sb, 0, st, (int)nv, rho,
                       0.0);
    if (pl.nproj > 0) hipLaunchKernelGGL(k_fill_f64, dim3(1), sb, 0, st, 3 * pl.nproj, dR, 0.0);
    PARO_HIP_TRY(hipGetLastError());
    // forward: step 1, then K outer iterations, keeping each Rayleigh-Ritz output
    auto ck_psi = [&](int n) { return a.ck_psi + (size_t)n * vstride; };
    auto ck_h = [&](int n) { return a.ck_h + (size_t)n * vstride; };
    auto ck_eps = [&](int n) { return a.ck_eps + (size_t)n * nb; };
    PARO_HIP_TRY(launch_copy_bands(st, nb, pl.ng, trial, ld, w.U, ldv));
    PARO_HIP_TRY(apply_full(pl, w, nb, w.U, ldv, w.W, nullptr));
    PARO_HIP_TRY(rayleigh_ritz(pl, w, nb, nb, w.U, w.W, ldv, ck_eps(0), ck_psi(0), ck_h(0), ldv));
    for (int n = 1; n <= K; ++n) {
        PARO_HIP_TRY(source_solve(pl, w, nb, ck_psi(n - 1), ck_h(n - 1), ldv, ck_eps(n - 1), w.sig_all, ncg, w.U, ldv,
                                  nullptr, 0));
        PARO_HIP_TRY(apply_full(pl, w, nb, w.U, ldv, w.W, nullptr));
        PARO_HIP_TRY(rayleigh_ritz(pl, w, nb, nb, w.U, w.W, ldv, ck_eps(n), ck_psi(n), ck_h(n), ldv));
    }
    hipLaunchKernelGGL(k_weighted_sum, dim3(1), sb, 0, st, nb, weights, ck_eps(K), energy);
    // backward
    hipLaunchKernelGGL(k_fill_c128, dim3(fg), sb, 0, st, nvec, a.psib);
    hipLaunchKernelGGL(k_fill_c128, dim3(fg), sb, 0, st, nvec, a.hb);
    PARO_HIP_TRY(hipMemcpyAsync(a.epsb, weights, sizeof(double) * nb, hipMemcpyDeviceToDevice, st));
    const dim3 vg = vgrid(pl, nb);
    for (int n = K; n >= 1; --n) {
        PARO_HIP_TRY(pcg_traced(pl, a, nb, ck_psi(n - 1), ck_h(n - 1), ck_eps(n - 1), ncg, w.U));
        PARO_HIP_TRY(apply_full(pl, w, nb, w.U, ldv, w.W, nullptr));
        PARO_HIP_TRY(rayleigh_ritz(pl, w, nb, nb, w.U, w.W, ldv, a.eps_t, a.psi_t, a.h_t, ldv));
        PARO_HIP_TRY(rr_backward(pl, a, nb, w.U, w.W, a.eps_t, a.psib, a.hb, a.epsb));
        PARO_HIP_TRY(apply_full(pl, w, nb, a.wb, ldv, a.tmp, nullptr));
        hipLaunchKernelGGL(k_axpy_bands, vg, dim3(kAdjThreads), 0, st, pl.ng, ldv, a.tmp, a.ub);
        PARO_HIP_TRY(accumulate_cross(pl, a, nb, a.wb, ldv, w.U, ldv, rho, dR));
        PARO_HIP_TRY(pcg_backward(pl, a, nb, ncg, ck_psi(n - 1), ck_eps(n - 1), rho, dR));
    }
    // step 1: Rayleigh-Ritz of the trial block (the trial block itself is fixed)
    PARO_HIP_TRY(launch_copy_bands(st, nb, pl.ng, trial, ld, w.U, ldv));
    PARO_HIP_TRY(apply_full(pl, w, nb, w.U, ldv, w.W, nullptr));
    PARO_HIP_TRY(rayleigh_ritz(pl, w, nb, nb, w.U, w.W, ldv, a.eps_t, a.psi_t, a.h_t, ldv));
    PARO_HIP_TRY(rr_backward(pl, a, nb, w.U, w.W, a.eps_t, a.psib, a.hb, a.epsb));
    PARO_HIP_TRY(accumulate_cross(pl, a, nb, a.wb, ldv, w.U, ldv, rho, dR));
    hipLaunchKernelGGL(k_scale_f64, dim3((unsigned)std::min<int64_t>((nv + 255) / 256, 65535)), sb, 0, st, nv,
                       1.0 / (double)nv, rho);
    PARO_HIP_TRY(hipStreamSynchronize(st));
    return PARO_OK;
}

}  // namespace

}  // namespace paro

using namespace paro;

extern "C" {

int32_t paro_truncated_gradient_workspace_bytes(paro_plan plan, int32_t nb, int32_t n_outer, int32_t n_cg,
                                                size_t *bytes)
{
    if (!plan || !bytes || nb <= 0 || nb > 1024 || n_outer < 1 || n_cg < 1) {
        set_error("paro_truncated_gradient_workspace_bytes: bad argument");
        return PARO_EINVAL;
    }
    *bytes = adj_layout(plan->pl, nb, n_outer, n_cg, nullptr, nullptr);
    return PARO_OK;
}

int32_t paro_truncated_gradient(paro_plan plan, int32_t nb, const double *trial, int64_t ld, double sigma,
                                int32_t n_outer, int32_t n_cg, const double *weights, double *energy, double *dvloc,
                                double *dR, void *ws, size_t ws_bytes)
{
    if (!plan || nb <= 0 || nb > 1024 || !trial || !weights || !energy || !dvloc || n_outer < 1 || n_cg < 1 || !ws ||
        !std::isfinite(sigma)) {
        set_error("paro_truncated_gradient: bad argument");
        return PARO_EINVAL;
    }
    const Plan &pl = plan->pl;
    if (ld < pl.ng) {
        set_error("paro_truncated_gradient: ld < n_g");
        return PARO_EINVAL;
    }
    if (pl.nproj > 0 && !dR) {
        set_error("paro_truncated_gradient: dR is NULL");
        return PARO_EINVAL;
    }
    if (big_grid(pl.grid[0])) {
        set_error("paro_truncated_gradient: grids above 96 points are not supported");
        return PARO_EUNSUP;
    }
    if (reinterpret_cast<uintptr_t>(ws) % 256) {
        set_error("paro_truncated_gradient: workspace must be 256-byte aligned");
        return PARO_EINVAL;
    }
    if (ws_bytes < adj_layout(pl, nb, n_outer, n_cg, nullptr, nullptr)) {
        set_error("paro_truncated_gradient: workspace smaller than paro_truncated_gradient_workspace_bytes");
        return PARO_ESIZE;
    }
    return truncated_gradient(pl, nb, (const double2 *)trial, ld, sigma, n_outer, n_cg, weights, energy, dvloc, dR,
                              ws);
}

}  // extern "C"
