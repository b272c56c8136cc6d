// Small dense FP64 linear algebra of the Rayleigh-Ritz step (Algorithm 1,
// step 4) on the GPU:  S = L L^H,  Hhat = L^-1 Hs L^-H,  Hhat = Q T Q^H
// (Householder, T real tridiagonal),  T = Z diag(lambda) Z^T (bisection on
// Sturm counts, then inverse iteration with Gram-Schmidt inside clusters),
// Y = Q Z,  C = L^-H Y.  Matrices are m x m column-major with ld = m.
// Everything runs in a few launches: one work-group for the factorisations
// that need the whole matrix, one wave per column for the triangular
// solves and the back-transformation.
#include <cfloat>
#include <cmath>

#include "group.h"
#include "paro_internal.h"
#include "reduce_device.h"

namespace paro {

namespace {

constexpr int kBig = 1024;

__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cmul_(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cjmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Hermitise S (first m columns of gram) into L and, when hs, Hs (next m
// columns) into X; then Cholesky of L in place (lower; upper zeroed).
// A pivot <= 1e-14 max_i S_ii sets fail[0] = 1 and the CHOL status bit.
__global__ void __launch_bounds__(kBig)
k_rr_chol(int m, const double2 *__restrict__ gram, int hs, double2 *__restrict__ L, double2 *__restrict__ X,
          int32_t *__restrict__ fail, int32_t *__restrict__ status)
{
    __shared__ double red[kBig / 64];
    __shared__ double s_ljj;
    __shared__ int s_fail;
    const int tid = threadIdx.x;
    const int64_t mm = (int64_t)m * m;
    double dmax = 0.0;
    for (int64_t e = tid; e < mm; e += kBig) {
        const int i = (int)(e % m), j = (int)(e / m);
        const double2 a = gram[e], b = gram[(int64_t)i * m + j];
        L[e] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
        if (i == j) dmax = fmax(dmax, a.x);
        if (hs) {
            const double2 c = gram[mm + e], d = gram[mm + (int64_t)i * m + j];
            X[e] = make_double2(0.5 * (c.x + d.x), 0.5 * (c.y - d.y));
        }
    }
    dmax = block_max<kBig>(dmax, red);
    if (tid == 0) s_fail = 0;
    __syncthreads();
    for (int j = 0; j < m; ++j) {
        if (tid == 0) {
            const double d = L[(int64_t)j * m + j].x;
            if (!(d > 1e-14 * dmax)) {
                s_fail = 1;
                s_ljj = 1.0;
            } else {
                s_ljj = sqrt(d);
            }
        }
        __syncthreads();
        if (s_fail) break;
        const double ljj = s_ljj, inv = 1.0 / ljj;
        for (int i = j + 1 + tid; i < m; i += kBig) {
            double2 v = L[(int64_t)j * m + i];
            L[(int64_t)j * m + i] = make_double2(v.x * inv, v.y * inv);
        }
        if (tid == 0) L[(int64_t)j * m + j] = make_double2(ljj, 0.0);
        __syncthreads();
        const int n = m - j - 1;
        for (int64_t e = tid; e < (int64_t)n * n; e += kBig) {
            const int il = (int)(e % n), ll = (int)(e / n);
            if (il < ll) continue;
            const int i = j + 1 + il, l = j + 1 + ll;
            const double2 a = L[(int64_t)j * m + i], b = L[(int64_t)j * m + l];
            double2 c = L[(int64_t)l * m + i];
            // c -= a conj(b)
            c.x -= a.x * b.x + a.y * b.y;
            c.y -= a.y * b.x - a.x * b.y;
            L[(int64_t)l * m + i] = c;
        }
        __syncthreads();
    }
    for (int64_t e = tid; e < mm; e += kBig) {
        const int i = (int)(e % m), j = (int)(e / m);
        if (i < j) L[e] = make_double2(0.0, 0.0);
    }
    if (tid == 0) {
        fail[0] = s_fail;
        if (s_fail) atomicOr(status, PARO_F_CHOL);
    }
}

// The same Cholesky by W wavefronts for m <= 64 R: lane l of every
// wavefront holds rows j + 1 + l + 64 r of the current column j (scaled by
// 1 / L_jj, computed identically by every wavefront, so no barrier is
// needed for the pivot); wavefront 0 writes the column back and to LDS; the
// columns of the trailing update are split over the wavefronts (columns
// j + 1 + wave, j + 1 + wave + W, ...), rows i >= l of column l.  Two
// barriers per column.  Dynamic LDS: m complex values.
template <int R, int W>
__device__ __forceinline__ void rr_chol_rows_body(int m, const double2 *__restrict__ gram, int hs,
                                                  double2 *__restrict__ L, double2 *__restrict__ X,
                                                  int32_t *__restrict__ fail, int32_t *__restrict__ status)
{
    __shared__ double red[W];
    extern __shared__ double2 sa[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int mm = m * m;
    double dmax = 0.0;
    for (int jj = wave; jj < m; jj += W)
        for (int ii = lane; ii < m; ii += 64) {
            const int q = jj * m + ii;
            const double2 a = gram[q], b = gram[ii * m + jj];
            L[q] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
            if (ii == jj) dmax = fmax(dmax, a.x);
            if (hs) {
                const double2 c = gram[mm + q], d = gram[mm + ii * m + jj];
                X[q] = make_double2(0.5 * (c.x + d.x), 0.5 * (c.y - d.y));
            }
        }
    dmax = block_max<64 * W>(dmax, red);  // ends with a barrier: L is complete
    int failed = 0;
    for (int j = 0; j < m; ++j) {
        const double dj = L[j * m + j].x;
        if (!(dj > 1e-14 * dmax)) {
            failed = 1;
            break;
        }
        const double ljj = sqrt(dj), inv = 1.0 / ljj;
        bool h[R];
        double2 a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = j + 1 + lane + 64 * r;
            h[r] = i < m;
            const double2 v = h[r] ? L[j * m + i] : make_double2(0.0, 0.0);
            a[r] = make_double2(v.x * inv, v.y * inv);
        }
        __syncthreads();  // every wavefront has read column j
        if (wave == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = j + 1 + lane + 64 * r;
                if (h[r]) L[j * m + i] = sa[i] = a[r];
            }
            if (lane == 0) L[j * m + j] = make_double2(ljj, 0.0);
        }
        __syncthreads();
        // L[i][l] -= L[i][j] conj(L[l][j]) for l > j, i >= l
#pragma unroll 4
        for (int l = j + 1 + wave; l < m; l += W) {
            const double2 b = sa[l];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = j + 1 + lane + 64 * r;
                if (h[r] && i >= l) {
                    double2 *c = L + l * m + i;
                    const double2 o = *c;
                    *c = make_double2(o.x - (a[r].x * b.x + a[r].y * b.y), o.y - (a[r].y * b.x - a[r].x * b.y));
                }
            }
        }
        __syncthreads();
    }
    __syncthreads();
    for (int jj = wave; jj < m; jj += W)
        for (int ii = lane; ii < jj; ii += 64) L[jj * m + ii] = make_double2(0.0, 0.0);
    if (tid == 0) {
        fail[0] = failed;
        if (failed) atomicOr(status, PARO_F_CHOL);
    }
}
template <int R, int W>
__global__ void __launch_bounds__(64 * W)
k_rr_chol_rows(int m, const double2 *__restrict__ gram, int hs, double2 *__restrict__ L, double2 *__restrict__ X,
               int32_t *__restrict__ fail, int32_t *__restrict__ status)
{
    rr_chol_rows_body<R, W>(m, gram, hs, L, X, fail, status);
}
// one work-group per entry
template <int R, int W> __global__ void __launch_bounds__(64 * W) k_rr_chol_rows_grp(GroupTab t)
{
    const CholArgs &a = *static_cast<const CholArgs *>(t.args[blockIdx.x]);
    rr_chol_rows_body<R, W>(a.m, a.gram, a.hs, a.L, a.X, a.fail, a.status);
}


// One column per single-wave work-group.
// mode 0: out = L^-1 b;  mode 1: out = L^-H b.
// b = column j of src, or (transb) the conjugate of row j of src.
__device__ __forceinline__ void trsm_col_body(int bx, int m, const double2 *__restrict__ L,
                                              const double2 *__restrict__ src, int transb, int mode,
                                              double2 *__restrict__ out)
{
    extern __shared__ double2 x[];
    const int j = bx, lane = threadIdx.x;
    for (int i = lane; i < m; i += 64)
        x[i] = transb ? cconj(src[(int64_t)i * m + j]) : src[(int64_t)j * m + i];
    __syncthreads();
    if (mode == 0) {
        for (int k = 0; k < m; ++k) {
            const double lkk = L[(int64_t)k * m + k].x;
            const double2 xk = make_double2(x[k].x / lkk, x[k].y / lkk);
            __syncthreads();
            if (lane == 0) x[k] = xk;
            for (int i = k + 1 + lane; i < m; i += 64) {
                const double2 l = L[(int64_t)k * m + i];
                const double2 t = cmul_(l, xk);
                x[i] = make_double2(x[i].x - t.x, x[i].y - t.y);
            }
            __syncthreads();
        }
    } else {
        for (int k = m - 1; k >= 0; --k) {
            const double lkk = L[(int64_t)k * m + k].x;
            const double2 xk = make_double2(x[k].x / lkk, x[k].y / lkk);
            __syncthreads();
            if (lane == 0) x[k] = xk;
            // x_i -= conj(L_ki) x_k for i < k; L_ki is row k of L: L[i*m + k]
            for (int i = lane; i < k; i += 64) {
                const double2 l = L[(int64_t)i * m + k];
                const double2 t = cjmul(l, xk);
                x[i] = make_double2(x[i].x - t.x, x[i].y - t.y);
            }
            __syncthreads();
        }
    }
    for (int i = lane; i < m; i += 64) out[(int64_t)j * m + i] = x[i];
}
__global__ void __launch_bounds__(64)
k_trsm_col(int m, const double2 *__restrict__ L, const double2 *__restrict__ src, int transb, int mode,
           double2 *__restrict__ out)
{
    trsm_col_body(blockIdx.x, m, L, src, transb, mode, out);
}
__global__ void __launch_bounds__(64) k_trsm_col_grp(GroupTab t)
{
    int e, bx, by;
    group_block(t, e, bx, by);
    const TrsmArgs &a = *static_cast<const TrsmArgs *>(t.args[e]);
    trsm_col_body(bx, a.m, a.L, a.src, a.transb, a.mode, a.out);
}


// Householder reduction of the Hermitian matrix A (hermitised first) to a
// real symmetric tridiagonal T = Q^H A Q, Q = H_0 ... H_{m-2},
// H_k = I - tau_k v_k v_k^H acting on rows k+1.., v_k[0] = 1, chosen so
// that H_k^H maps column k below the diagonal to (beta_k, 0, ...), beta_k
// real.  On exit: d (diagonal), e (off-diagonal, e_k = beta_k), tau, and
// v_k stored in column k of A below the diagonal.
//
// One work-group of kBig threads.  A (m x m, column-major, leading
// dimension m) is either the global matrix or a copy in LDS; sv, sy, sw
// (m each) and partial (kBig) are LDS scratch.
__device__ __forceinline__ void tridiag_run(int m, double2 *A, double *__restrict__ d, double *__restrict__ e,
                                            double2 *__restrict__ tau, double2 *sv, double2 *sy, double2 *sw,
                                            double2 *partial)
{
    __shared__ double red[kBig / 64];
    __shared__ double2 s_tau, s_scale;
    __shared__ double s_beta;
    const int tid = threadIdx.x;
    const int64_t mm = (int64_t)m * m;
    // hermitise in place (upper from lower average)
    for (int64_t q = tid; q < mm; q += kBig) {
        const int i = (int)(q % m), j = (int)(q / m);
        if (i > j) {
            const double2 a = A[q], b = A[(int64_t)i * m + j];
            const double2 h = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
            A[q] = h;
            A[(int64_t)i * m + j] = cconj(h);
        } else if (i == j) {
            A[q].y = 0.0;
        }
    }
    __syncthreads();
    for (int k = 0; k + 1 < m; ++k) {
        const int n = m - k - 1;
        double2 *col = A + (int64_t)k * m + k + 1;  // x = A[k+1:, k]
        double xn = 0.0;
        for (int i = 1 + tid; i < n; i += kBig) xn += col[i].x * col[i].x + col[i].y * col[i].y;
        xn = block_sum<kBig>(xn, red);
        if (tid == 0) {
            const double2 alpha = col[0];
            d[k] = A[(int64_t)k * m + k].x;
            if (xn == 0.0 && alpha.y == 0.0) {
                s_tau = make_double2(0.0, 0.0);
                s_beta = alpha.x;
                s_scale = make_double2(0.0, 0.0);
            } else {
                const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn);
                const double beta = alpha.x >= 0.0 ? -nrm : nrm;
                s_tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
                // scale = 1 / (alpha - beta)
                const double ar = alpha.x - beta, ai = alpha.y, den = ar * ar + ai * ai;
                s_scale = make_double2(ar / den, -ai / den);
                s_beta = beta;
            }
            e[k] = s_beta;
            tau[k] = s_tau;
        }
        __syncthreads();
        const double2 tk = s_tau, sc = s_scale;
        for (int i = tid; i < n; i += kBig) {
            const double2 v = i == 0 ? make_double2(1.0, 0.0) : cmul_(col[i], sc);
            sv[i] = v;
            col[i] = v;
        }
        __syncthreads();
        if (tk.x == 0.0 && tk.y == 0.0) continue;
        // y = A_trail v, A_trail = A[k+1:, k+1:]
        double2 *At = A + (int64_t)(k + 1) * m + k + 1;
        const int parts = kBig / n;
        const int i = tid % n, part = tid / n;
        if (part < parts) {
            const int jb = (int)((int64_t)n * part / parts), je = (int)((int64_t)n * (part + 1) / parts);
            double2 acc = make_double2(0.0, 0.0);
            for (int j = jb; j < je; ++j) {
                const double2 t = cmul_(At[(int64_t)j * m + i], sv[j]);
                acc.x += t.x;
                acc.y += t.y;
            }
            partial[part * n + i] = acc;
        }
        __syncthreads();
        double cr = 0.0;
        for (int r = tid; r < n; r += kBig) {
            double2 acc = make_double2(0.0, 0.0);
            for (int p = 0; p < parts; ++p) {
                acc.x += partial[p * n + r].x;
                acc.y += partial[p * n + r].y;
            }
            sy[r] = acc;
            const double2 c = cjmul(sv[r], acc);
            cr += c.x;
        }
        cr = block_sum<kBig>(cr, red);  // c = Re(v^H y)
        const double t2 = 0.5 * (tk.x * tk.x + tk.y * tk.y) * cr;
        for (int r = tid; r < n; r += kBig) {
            const double2 ty = cmul_(tk, sy[r]);
            sw[r] = make_double2(ty.x - t2 * sv[r].x, ty.y - t2 * sv[r].y);
        }
        __syncthreads();
        for (int64_t q = tid; q < (int64_t)n * n; q += kBig) {
            const int ii = (int)(q % n), jj = (int)(q / n);
            const double2 a = cjmul(sv[jj], sw[ii]);  // w_i conj(v_j)
            const double2 b = cjmul(sw[jj], sv[ii]);  // v_i conj(w_j)
            double2 c = At[(int64_t)jj * m + ii];
            c.x -= a.x + b.x;
            c.y -= a.y + b.y;
            At[(int64_t)jj * m + ii] = c;
        }
        __syncthreads();
    }
    if (tid == 0) {
        d[m - 1] = A[(int64_t)(m - 1) * m + m - 1].x;
        e[m - 1] = 0.0;
        tau[m - 1] = make_double2(0.0, 0.0);
    }
}

__global__ void __launch_bounds__(kBig)
k_tridiag(int m, double2 *__restrict__ A, double *__restrict__ d, double *__restrict__ e, double2 *__restrict__ tau)
{
    __shared__ double2 sv[kBig], sy[kBig], sw[kBig];
    __shared__ double2 partial[kBig];
    tridiag_run(m, A, d, e, tau, sv, sy, sw, partial);
}

// The same reduction by W wavefronts, the matrix either copied to LDS for
// the whole sweep (LDS, m <= kTridiagLdsMax) or updated in place in global
// memory (m <= 64 R).  Lane l of every wavefront holds rows l + 64 r
// (r < R) of the vectors x, v, y, w; the scalars of each Householder vector
// and the reductions over rows are computed redundantly and identically by
// every wavefront (shuffle trees, lane 0 broadcasts), so they need no
// barrier.  The column loops of y = A v and of the rank-2 update are split
// over the wavefronts (columns j = wave, wave + W, ...); the partial y of
// each wavefront is added in wavefront order.  Four work-group barriers
// per column.  In LDS eight wavefronts suffice; in global memory sixteen,
// with eight columns' loads in flight per wavefront, cover more of the
// cache latency of the column loops.  Dynamic LDS: (LDS ? m^2 : 0) +
// (2 + W) m complex values.
constexpr int kTriWavesLds = 8, kTriWavesGlobal = 16;
constexpr int kTriDistG = 16;  // work-groups of the multi-work-group tridiagonalisation
constexpr int kTridiagLdsMax = 92;
constexpr int kTridiagRowsMax = 5;  // rows per lane of the global-memory variant (m <= 320)
static size_t tridiag_lds_bytes(int m, bool lds)
{
    return sizeof(double2) * ((lds ? (size_t)m * m + (2 + kTriWavesLds) * (size_t)m
                                   : (2 + kTriWavesGlobal) * (size_t)m));
}

// sum over the wavefront (fixed shuffle tree), the same value in every lane
__device__ __forceinline__ double wave_sum_all(double v) { return __shfl(wave_sum(v), 0, 64); }

template <int R, bool LDS, int W>
__device__ __forceinline__ void tridiag_rows_body(int m, double2 *__restrict__ A, double *__restrict__ d,
                                                  double *__restrict__ e, double2 *__restrict__ tau)
{
    extern __shared__ double2 dyn[];
    double2 *S = LDS ? dyn : A;
    double2 *sv = LDS ? dyn + m * m : dyn, *sw = sv + m, *yp = sw + m;  // yp: W x m partial products
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NT = 64 * W;
    const int mm = m * m;
    if (LDS) {
        for (int q = tid; q < mm; q += NT) S[q] = A[q];
        __syncthreads();
    }
    // hermitise (upper from the average with the lower triangle)
    for (int jj = wave; jj < m; jj += W) {
        for (int ii = jj + 1 + lane; ii < m; ii += 64) {
            const double2 a = S[jj * m + ii], b = S[ii * m + jj];
            const double2 h = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
            S[jj * m + ii] = h;
            S[ii * m + jj] = cconj(h);
        }
        if (lane == 0) S[jj * m + jj].y = 0.0;
    }
    __syncthreads();
    for (int k = 0; k + 1 < m; ++k) {
        const int n = m - k - 1;
        double2 *col = S + k * m + k + 1;  // x = A[k+1:, k]
        bool h[R];
        double2 x[R], v[R], y[R], w[R];
        double xn = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = lane + 64 * r;
            h[r] = i < n;
            x[r] = h[r] ? col[i] : make_double2(0.0, 0.0);
            if (h[r] && i > 0) xn += x[r].x * x[r].x + x[r].y * x[r].y;
        }
        xn = wave_sum_all(xn);
        const double2 alpha = col[0];
        double2 tk, sc;
        double beta;
        if (xn == 0.0 && alpha.y == 0.0) {
            tk = make_double2(0.0, 0.0);
            beta = alpha.x;
            sc = make_double2(0.0, 0.0);
        } else {
            const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn);
            beta = alpha.x >= 0.0 ? -nrm : nrm;
            tk = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
            const double ar = alpha.x - beta, ai = alpha.y, den = ar * ar + ai * ai;
            sc = make_double2(ar / den, -ai / den);  // 1 / (alpha - beta)
        }
        const double dk = S[k * m + k].x;
        // v = x / (alpha - beta), v_0 = 1, kept in column k below the diagonal
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = lane + 64 * r;
            v[r] = h[r] ? (i == 0 ? make_double2(1.0, 0.0) : cmul_(x[r], sc)) : make_double2(0.0, 0.0);
        }
        __syncthreads();  // every wavefront has read column k
        if (wave == 0) {
            if (lane == 0) {
                d[k] = dk;
                e[k] = beta;
                tau[k] = tk;
            }
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (h[r]) col[lane + 64 * r] = sv[lane + 64 * r] = v[r];
        }
        __syncthreads();
        if (tk.x == 0.0 && tk.y == 0.0) continue;
        // partial y = A_trail v over this wavefront's columns, A_trail = A[k+1:, k+1:]
        double2 *At = S + (k + 1) * m + k + 1;
#pragma unroll
        for (int r = 0; r < R; ++r) y[r] = make_double2(0.0, 0.0);
#pragma unroll 8
        for (int jj = wave; jj < n; jj += W) {
            const double2 vj = sv[jj];
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (h[r]) {
                    const double2 t = cmul_(At[jj * m + lane + 64 * r], vj);
                    y[r].x += t.x;
                    y[r].y += t.y;
                }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (h[r]) yp[wave * m + lane + 64 * r] = y[r];
        __syncthreads();
        double crp = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            y[r] = make_double2(0.0, 0.0);
            if (h[r])
                for (int q = 0; q < W; ++q) {
                    y[r].x += yp[q * m + lane + 64 * r].x;
                    y[r].y += yp[q * m + lane + 64 * r].y;
                }
            crp += cjmul(v[r], y[r]).x;
        }
        // w = tau y - (|tau|^2 / 2) Re(v^H y) v
        const double cr = wave_sum_all(crp);
        const double t2 = 0.5 * (tk.x * tk.x + tk.y * tk.y) * cr;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double2 ty = cmul_(tk, y[r]);
            w[r] = make_double2(ty.x - t2 * v[r].x, ty.y - t2 * v[r].y);
        }
        if (wave == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (h[r]) sw[lane + 64 * r] = w[r];
        }
        __syncthreads();
        // A_trail -= w v^H + v w^H over this wavefront's columns
#pragma unroll 8
        for (int jj = wave; jj < n; jj += W) {
            const double2 vj = sv[jj], wj = sw[jj];
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (h[r]) {
                    const double2 a = cjmul(vj, w[r]), b = cjmul(wj, v[r]);  // w_i conj(v_j), v_i conj(w_j)
                    double2 *c = At + jj * m + lane + 64 * r;
                    const double2 o = *c;
                    *c = make_double2(o.x - (a.x + b.x), o.y - (a.y + b.y));
                }
        }
        __syncthreads();
    }
    if (tid == 0) {
        d[m - 1] = S[(m - 1) * m + m - 1].x;
        e[m - 1] = 0.0;
        tau[m - 1] = make_double2(0.0, 0.0);
    }
    if (LDS)
        for (int q = tid; q < mm; q += NT) A[q] = S[q];
}
template <int R, bool LDS, int W>
__global__ void __launch_bounds__(64 * W)
k_tridiag_rows(int m, double2 *__restrict__ A, double *__restrict__ d, double *__restrict__ e,
               double2 *__restrict__ tau)
{
    tridiag_rows_body<R, LDS, W>(m, A, d, e, tau);
}
// one work-group per entry
template <int R, bool LDS, int W> __global__ void __launch_bounds__(64 * W) k_tridiag_rows_grp(GroupTab t)
{
    const TridiagArgs &a = *static_cast<const TridiagArgs *>(t.args[blockIdx.x]);
    tridiag_rows_body<R, LDS, W>(a.m, a.A, a.d, a.e, a.tau);
}


// The same reduction with the matrix in registers (93 <= m <= 160): the
// matrix (409 KB at m = 160) fits neither LDS nor one compute unit's cache
// share, but it fits a 512-thread work-group's registers and LDS.  Thread
// (r, c) = (lane & 31, 2 wave + (lane >> 5)) holds A(i, j) for i = r + 32 a
// (a < 5) and j = c + 16 b (b < 10).  Rows 32 .. 159 (a >= 1) sit in
// registers (40 complex values, 160 registers per thread, indexed only
// with compile-time slots); rows 0 .. 31 (a = 0), which leave the trailing
// block after 31 columns, sit in LDS.  Per column k, three work-group
// barriers:
//   - the half-wavefront that holds column k forms the Householder vector
//     v (its norm summed over the half-wavefront) and publishes it in LDS
//     (two buffers, alternating with k) with tau;
//   - every thread sums y = A v over its columns for its rows; the two
//     halves of each wavefront are added, and each wavefront publishes its
//     partial y and its share of Re(v^H y);
//   - 160 threads add the partials in wavefront order and publish
//     w = tau y - (|tau|^2 / 2) Re(v^H y) v;
//   - every thread updates its own elements, A -= w v^H + v w^H.
// Entries outside the trailing block see v = w = 0 and stay unchanged.  The
// reflectors, d, e and tau go to global memory after the first barrier, so
// no barrier waits for a global store.  Dynamic LDS: kTriRegLds bytes.
constexpr int kTriRegMin = 93, kTriRegMax = 160, kTriRegWaves = 8;
constexpr int kTriRegA = 5, kTriRegB = 10;  // row and column slots per thread
static_assert(32 * kTriRegA >= kTriRegMax && 16 * kTriRegB >= kTriRegMax && 2 * kTriRegWaves == 16, "slots");
constexpr size_t kTriRegLds = sizeof(double2) * ((3 + kTriRegWaves) * kTriRegMax + 32 * kTriRegMax + 16);

// Cross-lane moves of a double without LDS: a DPP pattern inside each
// 16-lane row (two 32-bit moves), and the value of the lane 16 or 32 away
// (v_permlane16_swap / v_permlane32_swap with both operands the same: a
// lane with the distance bit clear finds its partner's value in the second
// result, the other lane in the first).
template <int CTRL> __device__ __forceinline__ double dpp_d(double v)
{
    uint32_t w[2];
    __builtin_memcpy(w, &v, sizeof(v));
#pragma unroll
    for (int h = 0; h < 2; ++h) w[h] = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w[h], CTRL, 0xf, 0xf, false);
    __builtin_memcpy(&v, w, sizeof(v));
    return v;
}
template <int D> __device__ __forceinline__ double lane_partner(double v)
{
    uint32_t w[2];
    __builtin_memcpy(w, &v, sizeof(v));
    const bool hi = threadIdx.x & D;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if constexpr (D == 16) {
            const auto r = __builtin_amdgcn_permlane16_swap(w[h], w[h], false, false);
            w[h] = hi ? r[0] : r[1];
        } else {
            const auto r = __builtin_amdgcn_permlane32_swap(w[h], w[h], false, false);
            w[h] = hi ? r[0] : r[1];
        }
    }
    __builtin_memcpy(&v, w, sizeof(v));
    return v;
}
// sum over the 32 lanes of each half-wavefront, the same value in each of
// them: lane pairs, quads (quad_perm), eights (row_half_mirror), rows
// (row_mirror), then the two rows of the half
__device__ __forceinline__ double half_sum(double v)
{
    v += dpp_d<0xb1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4e>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x141>(v);  // row_half_mirror
    v += dpp_d<0x140>(v);  // row_mirror
    return v + lane_partner<16>(v);
}
// Work-group barrier that waits for this wavefront's LDS accesses only,
// not for its global stores (a __syncthreads would hold every wavefront
// until the reflector stores of the column owner reached memory).  For
// data shared through LDS only; the compiler may not move memory accesses
// across it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}
// a double of one lane of the wavefront (uniform lane index)
__device__ __forceinline__ double lane_value(double v, int l)
{
    uint32_t w[2];
    __builtin_memcpy(w, &v, sizeof(v));
#pragma unroll
    for (int h = 0; h < 2; ++h) w[h] = (uint32_t)__builtin_amdgcn_readlane((int)w[h], l);
    __builtin_memcpy(&v, w, sizeof(v));
    return v;
}

__global__ void __launch_bounds__(64 * kTriRegWaves)
k_tridiag_reg(int m, double2 *__restrict__ A, double *__restrict__ d, double *__restrict__ e, double2 *__restrict__ tau)
{
    extern __shared__ double2 dyn[];
    double2 *vbuf = dyn;                            // v, two buffers of kTriRegMax
    double2 *ws = vbuf + 2 * kTriRegMax;
    double2 *part = ws + kTriRegMax;                // [wave][row]
    double2 *A0 = part + kTriRegWaves * kTriRegMax;  // rows 0 .. 31: A0[j * 32 + i]
    double2 *scal = A0 + 32 * kTriRegMax;           // tau (two buffers), Re(v^H y) per wavefront
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 31, c = 2 * wave + (lane >> 5);
    constexpr int NT = 64 * kTriRegWaves;
    // load, hermitised: A(i, j) <- (A(i, j) + conj(A(j, i))) / 2, real diagonal
    double2 a_[kTriRegA][kTriRegB];
#pragma unroll
    for (int a = 0; a < kTriRegA; ++a)
#pragma unroll
        for (int b = 0; b < kTriRegB; ++b) {
            const int i = r + 32 * a, j = c + 16 * b;
            double2 h = make_double2(0.0, 0.0);
            if (i < m && j < m) {
                const double2 x = A[(int64_t)j * m + i], y = A[(int64_t)i * m + j];
                h = i == j ? make_double2(x.x, 0.0) : make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
            }
            if (a == 0) A0[j * 32 + r] = h;
            else a_[a][b] = h;
        }
    __syncthreads();
    for (int k = 0; k + 1 < m; ++k) {
        const int n = m - k - 1;
        double2 *vs = vbuf + (k & 1) * kTriRegMax;
        // the half-wavefront holding column k: Householder vector and scalars
        double beta = 0.0, dk = 0.0;
        const bool owner = c == (k & 15);
        if (wave == ((k & 15) >> 1)) {
            double2 x[kTriRegA];
#pragma unroll
            for (int a = 0; a < kTriRegA; ++a) x[a] = make_double2(0.0, 0.0);
#pragma unroll
            for (int b = 0; b < kTriRegB; ++b)
                if (b == (k >> 4))
#pragma unroll
                    for (int a = 0; a < kTriRegA; ++a) x[a] = a == 0 ? A0[k * 32 + r] : a_[a][b];
            double xn = 0.0;
            double2 al = make_double2(0.0, 0.0);
#pragma unroll
            for (int a = 0; a < kTriRegA; ++a) {
                const int i = r + 32 * a;
                if (i > k + 1 && i < m) xn += x[a].x * x[a].x + x[a].y * x[a].y;
                if (a == ((k + 1) >> 5)) al = x[a];
                if (i == k) dk = x[a].x;
            }
            xn = half_sum(xn);
            // alpha = A(k + 1, k), from the owner lane of row k + 1
            const int la = ((k & 1) << 5) | ((k + 1) & 31);
            const double ar = lane_value(al.x, la), ai = lane_value(al.y, la);
            double2 tk, sc;
            if (xn == 0.0 && ai == 0.0) {
                tk = make_double2(0.0, 0.0);
                beta = ar;
                sc = make_double2(0.0, 0.0);
            } else {
                const double nrm = sqrt(ar * ar + ai * ai + xn);
                beta = ar >= 0.0 ? -nrm : nrm;
                tk = make_double2((beta - ar) / beta, -ai / beta);
                const double br = ar - beta, den = br * br + ai * ai;
                sc = make_double2(br / den, -ai / den);  // 1 / (alpha - beta)
            }
#pragma unroll
            for (int a = 0; a < kTriRegA; ++a) {
                const int i = r + 32 * a;
                const double2 v = i == k + 1 ? make_double2(1.0, 0.0)
                                             : (i > k + 1 && i < m ? cmul_(x[a], sc) : make_double2(0.0, 0.0));
                if (owner) vs[i] = v;
            }
            if (owner && r == 0) scal[k & 1] = tk;
        }
        lds_barrier();
        const double2 tk = scal[k & 1];
        if (owner && wave == ((k & 15) >> 1)) {
            // the reflector (below the diagonal of column k) and the scalars
#pragma unroll
            for (int a = 0; a < kTriRegA; ++a) {
                const int i = r + 32 * a;
                if (i > k && i < m) A[(int64_t)k * m + i] = vs[i];
                if (i == k) d[k] = dk;
            }
            if (r == 0) {
                e[k] = beta;
                tau[k] = tk;
            }
        }
        if (tk.x == 0.0 && tk.y == 0.0) continue;
        // partial y over this thread's columns (column slots outer: each v_j
        // is read once), then over the two half-waves; this wavefront's share
        // of Re(v^H y)
        double2 acc[kTriRegA];
#pragma unroll
        for (int a = 0; a < kTriRegA; ++a) acc[a] = make_double2(0.0, 0.0);
#pragma unroll
        for (int b = 0; b < kTriRegB; ++b) {
            if (16 * b + 15 <= k || 16 * b >= m) continue;
            const int j = c + 16 * b;
            const double2 vj = vs[j];
#pragma unroll
            for (int a = 0; a < kTriRegA; ++a) {
                if (32 * a + 31 <= k || 32 * a >= m) continue;
                const double2 t = cmul_(a == 0 ? A0[j * 32 + r] : a_[a][b], vj);
                acc[a].x += t.x;
                acc[a].y += t.y;
            }
        }
        double crp = 0.0;
#pragma unroll
        for (int a = 0; a < kTriRegA; ++a) {
            if (32 * a + 31 <= k || 32 * a >= m) continue;
            acc[a].x += lane_partner<32>(acc[a].x);
            acc[a].y += lane_partner<32>(acc[a].y);
            const int i = r + 32 * a;
            if (i > k && i < m) {
                if (lane < 32) part[wave * kTriRegMax + i] = acc[a];
                crp += cjmul(vs[i], acc[a]).x;
            }
        }
        crp = half_sum(crp);
        if (lane == 0) scal[2 + wave].x = crp;
        lds_barrier();
        // y over the wavefronts, in wavefront order, and w = tau y - (|tau|^2 / 2) Re(v^H y) v
        double cr = 0.0;
#pragma unroll
        for (int q = 0; q < kTriRegWaves; ++q) cr += scal[2 + q].x;
        const double t2 = 0.5 * (tk.x * tk.x + tk.y * tk.y) * cr;
        for (int i = tid; i < kTriRegMax; i += NT) {
            double2 y = make_double2(0.0, 0.0);
            if (i > k && i < m)
#pragma unroll
                for (int q = 0; q < kTriRegWaves; ++q) {
                    y.x += part[q * kTriRegMax + i].x;
                    y.y += part[q * kTriRegMax + i].y;
                }
            const double2 ty = cmul_(tk, y), v = vs[i];
            ws[i] = make_double2(ty.x - t2 * v.x, ty.y - t2 * v.y);
        }
        lds_barrier();
        // A -= w v^H + v w^H on this thread's elements (column slots outer:
        // v_j, w_j read once; v_i, w_i of the five row slots held throughout)
        double2 vi[kTriRegA], wi[kTriRegA];
#pragma unroll
        for (int a = 0; a < kTriRegA; ++a) {
            vi[a] = vs[r + 32 * a];
            wi[a] = ws[r + 32 * a];
        }
#pragma unroll
        for (int b = 0; b < kTriRegB; ++b) {
            if (16 * b + 15 <= k || 16 * b >= m) continue;
            const int j = c + 16 * b;
            const double2 vj = vs[j], wj = ws[j];
#pragma unroll
            for (int a = 0; a < kTriRegA; ++a) {
                if (32 * a + 31 <= k || 32 * a >= m) continue;
                const double2 p = cjmul(vj, wi[a]), q = cjmul(wj, vi[a]);  // w_i conj(v_j), v_i conj(w_j)
                if (a == 0) {
                    double2 &o = A0[j * 32 + r];
                    o = make_double2(o.x - (p.x + q.x), o.y - (p.y + q.y));
                } else {
                    a_[a][b].x -= p.x + q.x;
                    a_[a][b].y -= p.y + q.y;
                }
            }
        }
    }
    // last diagonal element (row m - 1 >= 92 lies in the register rows)
#pragma unroll
    for (int a = 1; a < kTriRegA; ++a)
#pragma unroll
        for (int b = 0; b < kTriRegB; ++b)
            if (r + 32 * a == m - 1 && c + 16 * b == m - 1) {
                d[m - 1] = a_[a][b].x;
                e[m - 1] = 0.0;
                tau[m - 1] = make_double2(0.0, 0.0);
            }
}

// Cholesky of the hermitised S (and hermitised Hs into X when hs) with the
// matrix in registers, 93 <= m <= 160, in the layout of k_tridiag_reg:
// thread (r, c) holds S(r + 32 a, c + 16 b), rows 32 .. 159 in registers,
// rows 0 .. 31 in LDS.  One work-group barrier per column: the half-
// wavefront that holds column j checks the pivot, forms the column of L
// (l_i = S(i, j) / sqrt(S(j, j)), i > j), publishes it in LDS (two buffers,
// alternating with j) and writes column j of L (zero above the diagonal);
// after the barrier every thread updates its trailing elements on or below
// the diagonal, S(i, l) -= l_i conj(l_l), and the holder of column j + 1
// goes on at once.
// A pivot at or below 1e-14 max_i S(i, i) stops the factorisation and sets
// fail and PARO_F_CHOL, as the other Cholesky kernels do.
constexpr size_t kCholRegLds = sizeof(double2) * (2 * kTriRegMax + 32 * kTriRegMax) + sizeof(double) * (kTriRegWaves + 1);

__global__ void __launch_bounds__(64 * kTriRegWaves)
k_chol_reg(int m, const double2 *__restrict__ gram, int hs, double2 *__restrict__ L, double2 *__restrict__ X,
           int32_t *__restrict__ fail, int32_t *__restrict__ status)
{
    extern __shared__ double2 dyn[];
    double2 *lbuf = dyn;                   // the current column of L, two buffers
    double2 *A0 = lbuf + 2 * kTriRegMax;   // rows 0 .. 31: A0[j * 32 + i]
    double *red = reinterpret_cast<double *>(A0 + 32 * kTriRegMax);  // kTriRegWaves maxima, then the stop flag
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 31, c = 2 * wave + (lane >> 5);
    constexpr int NT = 64 * kTriRegWaves;
    const int64_t mm = (int64_t)m * m;
    // the hermitised Hs to X (rows in lanes: coalesced stores)
    if (hs)
        for (int64_t q = tid; q < mm; q += NT) {
            const int jj = (int)(q / m), ii = (int)(q - (int64_t)jj * m);
            const double2 a = gram[mm + q], b = gram[mm + (int64_t)ii * m + jj];
            X[q] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
        }
    // the hermitised S, and the largest diagonal element
    double2 a_[kTriRegA][kTriRegB];
    double dmax = 0.0;
#pragma unroll
    for (int a = 0; a < kTriRegA; ++a)
#pragma unroll
        for (int b = 0; b < kTriRegB; ++b) {
            const int i = r + 32 * a, j = c + 16 * b;
            double2 h = make_double2(0.0, 0.0);
            if (i < m && j < m) {
                const double2 x = gram[(int64_t)j * m + i], y = gram[(int64_t)i * m + j];
                h = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
                if (i == j) dmax = fmax(dmax, x.x);
            }
            if (a == 0) A0[j * 32 + r] = h;
            else a_[a][b] = h;
        }
    dmax = wave_max(dmax);
    if (lane == 0) red[wave] = dmax;
    if (tid == 0) red[kTriRegWaves] = 0.0;
    __syncthreads();
    dmax = red[0];
#pragma unroll
    for (int q = 1; q < kTriRegWaves; ++q) dmax = fmax(dmax, red[q]);
    int failed = 0, jf = m;
    for (int j = 0; j < m; ++j) {
        double2 *ls = lbuf + (j & 1) * kTriRegMax;
        if (c == (j & 15)) {
            // the half-wavefront holding column j
            double2 x[kTriRegA];
#pragma unroll
            for (int a = 0; a < kTriRegA; ++a) x[a] = make_double2(0.0, 0.0);
#pragma unroll
            for (int b = 0; b < kTriRegB; ++b)
                if (b == (j >> 4))
#pragma unroll
                    for (int a = 0; a < kTriRegA; ++a) x[a] = a == 0 ? A0[j * 32 + r] : a_[a][b];
            double dl = 0.0;
#pragma unroll
            for (int a = 0; a < kTriRegA; ++a)
                if (a == (j >> 5)) dl = x[a].x;
            const double dj = lane_value(dl, ((j & 1) << 5) | (j & 31));
            if (!(dj > 1e-14 * dmax)) {
                if (r == 0) red[kTriRegWaves] = 1.0;
            } else {
                const double ljj = sqrt(dj), inv = 1.0 / ljj;
#pragma unroll
                for (int a = 0; a < kTriRegA; ++a) {
                    const int i = r + 32 * a;
                    const double2 l = i > j && i < m ? make_double2(x[a].x * inv, x[a].y * inv)
                                                     : make_double2(0.0, 0.0);
                    ls[i] = l;
                    if (i < m) L[(int64_t)j * m + i] = i == j ? make_double2(ljj, 0.0) : l;
                }
            }
        }
        lds_barrier();
        if (red[kTriRegWaves] != 0.0) {
            failed = 1;
            jf = j;
            break;
        }
        // S(i, l) -= l_i conj(l_l) on the trailing elements
        double2 li[kTriRegA];
#pragma unroll
        for (int a = 0; a < kTriRegA; ++a) li[a] = ls[r + 32 * a];
#pragma unroll
        for (int b = 0; b < kTriRegB; ++b) {
            if (16 * b + 15 <= j || 16 * b >= m) continue;
            const double2 ll = ls[c + 16 * b];
#pragma unroll
            for (int a = 0; a < kTriRegA; ++a) {
                // trailing slots on or below the diagonal only (the upper triangle is never read)
                if (32 * a + 31 <= j || 32 * a >= m || 16 * b > 32 * a + 31) continue;
                const double2 p = cjmul(ll, li[a]);  // l_i conj(l_l)
                if (a == 0) {
                    double2 &o = A0[(c + 16 * b) * 32 + r];
                    o = make_double2(o.x - p.x, o.y - p.y);
                } else {
                    a_[a][b].x -= p.x;
                    a_[a][b].y -= p.y;
                }
            }
        }
    }
    if (failed) {
        // the columns not factorised keep the partly updated lower triangle
#pragma unroll
        for (int a = 0; a < kTriRegA; ++a)
#pragma unroll
            for (int b = 0; b < kTriRegB; ++b) {
                const int i = r + 32 * a, l = c + 16 * b;
                if (i < m && l < m && l >= jf) {
                    const double2 v = a == 0 ? A0[l * 32 + r] : a_[a][b];
                    L[(int64_t)l * m + i] = i >= l ? v : make_double2(0.0, 0.0);
                }
            }
    }
    if (tid == 0) {
        fail[0] = failed;
        if (failed) atomicOr(status, PARO_F_CHOL);
    }
}

// The same reduction spread over G work-groups (G = 16 for 208 <= m <= 352,
// G = 64 for 352 < m <= 704),
// each holding the columns c = g, g + G, ... of the hermitised matrix in
// its LDS for the whole sweep, so that the trailing updates read and write
// LDS only.  Per column k: the owner of column k forms the Householder
// vector and publishes it (with tau) in a global buffer behind a flag;
// every work-group that owns a trailing column forms the partial
// y = A v over its own columns and publishes it behind a counter; each then
// adds the partials in work-group order, forms w and updates its own
// columns.  The buffers alternate between even and odd columns: a buffer is
// rewritten two columns later, after every reader has passed the next
// column's exchange.  Every wait has a time limit; a work-group that
// reaches it raises a global abort flag that ends every other wait, and
// sets PARO_F_SYNC.  The G work-groups are launched as an ordinary
// grid after a check that one fits on a compute unit (dist_grid_fits):
// with 16 or 64 of them on a 256-unit device they start together, and a
// work-group held back by other kernels' work-groups starts once those
// end, so every wait either succeeds or reaches its limit.  Dynamic LDS:
// (ceil(m / G) + 2) m + 1 complex values.
constexpr int kTriDistThreads = 256;
constexpr int kTriDistMin = 93, kTriDistMax = 352;
// The second size class: 64 work-groups of 512 threads for 352 < m <= 704
// (m = 704: 11 columns per work-group, (11 + 2) 704 complex = 146 KB of LDS;
// 512 threads cover the 2 x 512 rows the tridiagonalisation's y and w
// loops take per thread).
constexpr int kTriDistG2 = 64, kTriDistThreads2 = 512, kTriDistMax2 = 704;
// The tridiagonalisation moves to sixteen work-groups only from m = 208:
// below that the one-work-group sweep is faster (m = 160: 1.7 against
// 2.0 ms per eigendecomposition; m = 192: 2.3 against 2.5; m = 256: 4.3
// against 3.5).  The Cholesky gains from m = 93 on.
constexpr int kTriDistMinTridiag = 208;
constexpr long long kTriDistWaitTicks = 20000000;  // 0.2 s of the 100 MHz real-time counter

template <int G> static size_t tridiag_dist_lds_bytes(int m)
{
    return sizeof(double2) * (((size_t)(m + G - 1) / G + 2) * (size_t)m + 1);
}
template <int G> static size_t chol_dist_lds_bytes(int m)
{
    return sizeof(double2) * (((size_t)(m + G - 1) / G + 1) * (size_t)m);
}

// wait until *p >= target (thread 0 of the work-group); false on abort or time-out
__device__ bool dist_wait(const int32_t *p, int target, int32_t *abortf, int32_t *status)
{
    const long long t0 = (long long)__builtin_amdgcn_s_memrealtime();
    for (;;) {
        if (__hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= target) return true;
        if (__hip_atomic_load(abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
        if ((long long)__builtin_amdgcn_s_memrealtime() - t0 > kTriDistWaitTicks) {
            __hip_atomic_store(abortf, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (status) atomicOr(status, PARO_F_SYNC);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

template <int G, int NT>
__global__ void __launch_bounds__(NT)
k_tridiag_dist(int m, double2 *__restrict__ A, double *__restrict__ d, double *__restrict__ e,
               double2 *__restrict__ tau, double2 *__restrict__ vbuf, double2 *__restrict__ ypart,
               int32_t *__restrict__ flags, int32_t *__restrict__ status)
{
    extern __shared__ double2 dyn[];
    __shared__ double red[NT / 64];
    __shared__ int s_ok;
    const int g = blockIdx.x, tid = threadIdx.x;
    const int nl = (m - g + G - 1) / G;  // own columns c = g + G s, s < nl
    // sv: v (and tau in slot m), sw: w
    double2 *loc = dyn, *sv = loc + (size_t)((m + G - 1) / G) * m, *sw = sv + m + 1;
    int32_t *vflag = flags, *ycnt = flags + m, *abortf = flags + 2 * m;
    // own columns of the hermitised matrix: h_ic = (A_ic + conj(A_ci)) / 2, real diagonal
    for (int sidx = 0; sidx < nl; ++sidx) {
        const int c = g + G * sidx;
        for (int i = tid; i < m; i += NT) {
            const double2 a = A[(size_t)c * m + i], b = A[(size_t)i * m + c];
            loc[(size_t)sidx * m + i] =
                i == c ? make_double2(a.x, 0.0) : make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
        }
    }
    __syncthreads();
    bool ok = true;
    for (int k = 0; k + 1 < m && ok; ++k) {
        const int n = m - k - 1;
        double2 *vb = vbuf + (size_t)(k & 1) * (m + 1);
        double2 *yb = ypart + (size_t)(k & 1) * G * m;
        if (g == k % G) {
            double2 *col = loc + (size_t)(k / G) * m;
            double xn = 0.0;
            for (int i = k + 2 + tid; i < m; i += NT) xn += col[i].x * col[i].x + col[i].y * col[i].y;
            xn = block_sum<NT>(xn, red);
            const double2 alpha = col[k + 1];
            double2 tk, sc;
            double beta;
            if (xn == 0.0 && alpha.y == 0.0) {
                tk = make_double2(0.0, 0.0);
                beta = alpha.x;
                sc = make_double2(0.0, 0.0);
            } else {
                const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn);
                beta = alpha.x >= 0.0 ? -nrm : nrm;
                tk = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
                const double ar = alpha.x - beta, ai = alpha.y, den = ar * ar + ai * ai;
                sc = make_double2(ar / den, -ai / den);  // 1 / (alpha - beta)
            }
            for (int i = k + 1 + tid; i < m; i += NT) {
                const double2 v = i == k + 1 ? make_double2(1.0, 0.0) : cmul_(col[i], sc);
                col[i] = v;
                vb[i] = v;
            }
            if (tid == 0) {
                d[k] = col[k].x;
                e[k] = beta;
                tau[k] = tk;
                vb[m] = tk;
            }
            __syncthreads();
            if (tid == 0) {
                __threadfence();
                __hip_atomic_store(&vflag[k], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (g + G * (nl - 1) <= k) break;  // no own column after k: this work-group is done
        if (tid == 0) s_ok = dist_wait(&vflag[k], 1, abortf, status) ? 1 : 0;
        __syncthreads();
        if (!s_ok) {
            ok = false;
            break;
        }
        for (int i = k + 1 + tid; i <= m; i += NT) sv[i] = vb[i];  // v and, in slot m, tau
        __syncthreads();
        const double2 tk = sv[m];
        if (tk.x == 0.0 && tk.y == 0.0) {
            __syncthreads();
            continue;
        }
        // partial y = sum over own columns c > k of A[:, c] v_c, rows k+1 .. m-1
        const int i0 = k + 1 + tid, i1 = i0 + NT;
        double2 y0 = make_double2(0.0, 0.0), y1 = make_double2(0.0, 0.0);
        for (int sidx = (k + 1 - g + G - 1) / G; sidx < nl; ++sidx) {
            const int c = g + G * sidx;
            const double2 vc = sv[c];
            const double2 *lc = loc + (size_t)sidx * m;
            if (i0 < m) {
                const double2 t = cmul_(lc[i0], vc);
                y0.x += t.x;
                y0.y += t.y;
            }
            if (i1 < m) {
                const double2 t = cmul_(lc[i1], vc);
                y1.x += t.x;
                y1.y += t.y;
            }
        }
        if (i0 < m) yb[(size_t)g * m + i0] = y0;
        if (i1 < m) yb[(size_t)g * m + i1] = y1;
        __syncthreads();
        if (tid == 0) {
            __threadfence();
            __hip_atomic_fetch_add(&ycnt[k], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            s_ok = dist_wait(&ycnt[k], n < G ? n : G, abortf, status) ? 1 : 0;
        }
        __syncthreads();
        if (!s_ok) {
            ok = false;
            break;
        }
        // y: the partials of the work-groups that own a column after k, in work-group order
        y0 = y1 = make_double2(0.0, 0.0);
        for (int q = 0; q < G; ++q) {
            if (n < G && ((q - (k + 1)) % G + G) % G >= n) continue;
            if (i0 < m) {
                const double2 t = yb[(size_t)q * m + i0];
                y0.x += t.x;
                y0.y += t.y;
            }
            if (i1 < m) {
                const double2 t = yb[(size_t)q * m + i1];
                y1.x += t.x;
                y1.y += t.y;
            }
        }
        const double2 v0 = i0 < m ? sv[i0] : make_double2(0.0, 0.0);
        const double2 v1 = i1 < m ? sv[i1] : make_double2(0.0, 0.0);
        // w = tau y - (|tau|^2 / 2) Re(v^H y) v
        const double cr = block_sum<NT>(cjmul(v0, y0).x + cjmul(v1, y1).x, red);
        const double t2 = 0.5 * (tk.x * tk.x + tk.y * tk.y) * cr;
        if (i0 < m) {
            const double2 ty = cmul_(tk, y0);
            sw[i0] = make_double2(ty.x - t2 * v0.x, ty.y - t2 * v0.y);
        }
        if (i1 < m) {
            const double2 ty = cmul_(tk, y1);
            sw[i1] = make_double2(ty.x - t2 * v1.x, ty.y - t2 * v1.y);
        }
        __syncthreads();
        // own columns c > k: A[:, c] -= w conj(v_c) + v conj(w_c)
        for (int sidx = (k + 1 - g + G - 1) / G; sidx < nl; ++sidx) {
            const int c = g + G * sidx;
            const double2 vc = sv[c], wc = sw[c];
            double2 *lc = loc + (size_t)sidx * m;
            if (i0 < m) {
                const double2 a = cjmul(vc, sw[i0]), b = cjmul(wc, v0);
                lc[i0] = make_double2(lc[i0].x - (a.x + b.x), lc[i0].y - (a.y + b.y));
            }
            if (i1 < m) {
                const double2 a = cjmul(vc, sw[i1]), b = cjmul(wc, v1);
                lc[i1] = make_double2(lc[i1].x - (a.x + b.x), lc[i1].y - (a.y + b.y));
            }
        }
        __syncthreads();
    }
    // own columns back to global memory (the Householder vectors below the diagonal)
    for (int sidx = 0; sidx < nl; ++sidx) {
        const int c = g + G * sidx;
        for (int i = tid; i < m; i += NT) A[(size_t)c * m + i] = loc[(size_t)sidx * m + i];
    }
    if (g == (m - 1) % G && tid == 0) {
        d[m - 1] = loc[(size_t)((m - 1) / G) * m + m - 1].x;
        e[m - 1] = 0.0;
        tau[m - 1] = make_double2(0.0, 0.0);
    }
}

__global__ void __launch_bounds__(256) k_fill_i32(int n, int32_t *__restrict__ p, int32_t v)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = v;
}

// The same Cholesky spread over G work-groups (G = 16 for 92 < m <= 352,
// G = 64 for 352 < m <= 704),
// each holding the columns c = g, g + G, ... of the hermitised S in its LDS
// for the whole factorisation.  Per column j the owner checks the pivot,
// scales its column, writes it (final) to L in global memory and raises
// the column's flag (2: the pivot failed); every work-group with a column
// after j waits for the flag, reads column j of L and updates its own
// columns.  Published columns are final, so no buffer is reused.  Waits
// are time-limited as in k_tridiag_dist, and the launch is the same
// ordinary grid.  Dynamic LDS: (ceil(m / G) + 1) m complex values.
template <int G, int NT>
__global__ void __launch_bounds__(NT)
k_chol_dist(int m, const double2 *__restrict__ gram, int hs, double2 *__restrict__ L, double2 *__restrict__ X,
            int32_t *__restrict__ flags, int32_t *__restrict__ fail, int32_t *__restrict__ status)
{
    extern __shared__ double2 dyn[];
    __shared__ double red[NT / 64];
    __shared__ int s_state;
    const int g = blockIdx.x, tid = threadIdx.x;
    const int nl = (m - g + G - 1) / G;
    double2 *loc = dyn, *sa = loc + (size_t)((m + G - 1) / G) * m;
    int32_t *cflag = flags, *abortf = flags + 2 * m;
    const size_t mm = (size_t)m * m;
    double dmax = 0.0;
    for (int i = tid; i < m; i += NT) dmax = fmax(dmax, gram[(size_t)i * m + i].x);
    dmax = block_max<NT>(dmax, red);
    for (int sidx = 0; sidx < nl; ++sidx) {
        const int c = g + G * sidx;
        for (int i = tid; i < m; i += NT) {
            const double2 a = gram[(size_t)c * m + i], b = gram[(size_t)i * m + c];
            loc[(size_t)sidx * m + i] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
            if (hs) {
                const double2 x = gram[mm + (size_t)c * m + i], y = gram[mm + (size_t)i * m + c];
                X[(size_t)c * m + i] = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
            }
        }
    }
    __syncthreads();
    for (int j = 0; j < m; ++j) {
        if (g == j % G) {
            double2 *col = loc + (size_t)(j / G) * m;
            const double dj = col[j].x;
            const bool bad = !(dj > 1e-14 * dmax);
            if (!bad) {
                const double ljj = sqrt(dj), inv = 1.0 / ljj;
                for (int i = j + 1 + tid; i < m; i += NT) {
                    const double2 v = make_double2(col[i].x * inv, col[i].y * inv);
                    col[i] = v;
                    L[(size_t)j * m + i] = v;
                }
                if (tid == 0) {
                    col[j] = make_double2(ljj, 0.0);
                    L[(size_t)j * m + j] = col[j];
                }
            }
            __syncthreads();
            if (tid == 0) {
                __threadfence();
                __hip_atomic_store(&cflag[j], bad ? 2 : 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                if (bad) {
                    fail[0] = 1;
                    atomicOr(status, PARO_F_CHOL);
                }
            }
            if (bad) break;
        }
        if (g + G * (nl - 1) <= j) break;  // no own column after j
        if (tid == 0) {
            s_state = dist_wait(&cflag[j], 1, abortf, status) ? 1 : 0;
            if (s_state && __hip_atomic_load(&cflag[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 2)
                s_state = 0;
        }
        __syncthreads();
        if (!s_state) break;
        for (int i = j + 1 + tid; i < m; i += NT) sa[i] = L[(size_t)j * m + i];
        __syncthreads();
        // own columns l > j, rows i >= l: L_il -= L_ij conj(L_lj)
        for (int sidx = (j + 1 - g + G - 1) / G; sidx < nl; ++sidx) {
            const int l = g + G * sidx;
            const double2 b = sa[l];
            double2 *lc = loc + (size_t)sidx * m;
            for (int i = l + tid; i < m; i += NT) {
                const double2 a = sa[i];
                lc[i] = make_double2(lc[i].x - (a.x * b.x + a.y * b.y), lc[i].y - (a.y * b.x - a.x * b.y));
            }
        }
        __syncthreads();
    }
    // own columns: zero above the diagonal; columns not yet published (after
    // a stop) are written as they stand
    for (int sidx = 0; sidx < nl; ++sidx) {
        const int c = g + G * sidx;
        for (int i = tid; i < c; i += NT) L[(size_t)c * m + i] = make_double2(0.0, 0.0);
        if (__hip_atomic_load(&cflag[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 1)
            for (int i = c + tid; i < m; i += NT) L[(size_t)c * m + i] = loc[(size_t)sidx * m + i];
    }
}

// Whether the G work-groups of NT threads of a multi-work-group dense kernel
// can be resident at once: at least one work-group with `lds` bytes of
// dynamic LDS fits on a compute unit, and the device has at least G units.
// Checked once per kernel and size class.
static bool dist_grid_fits(const void *kernel, int G, int NT, size_t lds)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, NT, lds) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return per_cu >= 1 && cus >= G;
}

// One size class of the multi-work-group Cholesky: set up once, then
// launched for kTriDistMin <= m <= MMAX.
template <int G, int NT, int MMAX>
static bool launch_chol_dist(hipStream_t st, int m, const double2 *gram, int hs, double2 *L, double2 *X,
                             int32_t *fail, int32_t *status, int32_t *flags)
{
    const void *k = reinterpret_cast<const void *>(k_chol_dist<G, NT>);
    static const bool ok = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)chol_dist_lds_bytes<G>(MMAX)) == hipSuccess &&
                           dist_grid_fits(k, G, NT, chol_dist_lds_bytes<G>(MMAX));
    if (!ok) return false;
    hipLaunchKernelGGL(k_fill_i32, dim3((2 * m + 1 + 255) / 256), dim3(256), 0, st, 2 * m + 1, flags, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, st, 1, fail, 0);
    hipLaunchKernelGGL((k_chol_dist<G, NT>), dim3(G), dim3(NT), chol_dist_lds_bytes<G>(m), st, m, gram, hs, L, X,
                       flags, fail, status);
    return true;
}

// Cholesky of the hermitised S (and hermitised Hs into X when hs): the
// row-held variant up to m = 320, the first design beyond.
static void launch_chol(hipStream_t st, int m, const double2 *gram, int hs, double2 *L, double2 *X, int32_t *fail,
                        int32_t *status, int32_t *flags = nullptr)
{
    static const hipError_t reg_attr = hipFuncSetAttribute(reinterpret_cast<const void *>(k_chol_reg),
                                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCholRegLds);
    if (m >= kTriRegMin && m <= kTriRegMax && reg_attr == hipSuccess) {
        hipLaunchKernelGGL(k_chol_reg, dim3(1), dim3(64 * kTriRegWaves), kCholRegLds, st, m, gram, hs, L, X, fail,
                           status);
        return;
    }
    if (flags && m >= kTriDistMin && m <= kTriDistMax &&
        launch_chol_dist<kTriDistG, kTriDistThreads, kTriDistMax>(st, m, gram, hs, L, X, fail, status, flags))
        return;
    if (flags && m > kTriDistMax && m <= kTriDistMax2 &&
        launch_chol_dist<kTriDistG2, kTriDistThreads2, kTriDistMax2>(st, m, gram, hs, L, X, fail, status, flags))
        return;
    constexpr int W = 16;
    const size_t sh = sizeof(double2) * (size_t)m;
    const dim3 tb(64 * W);
    if (m <= 128)
        hipLaunchKernelGGL((k_rr_chol_rows<2, W>), dim3(1), tb, sh, st, m, gram, hs, L, X, fail, status);
    else if (m <= 192)
        hipLaunchKernelGGL((k_rr_chol_rows<3, W>), dim3(1), tb, sh, st, m, gram, hs, L, X, fail, status);
    else if (m <= 256)
        hipLaunchKernelGGL((k_rr_chol_rows<4, W>), dim3(1), tb, sh, st, m, gram, hs, L, X, fail, status);
    else if (m <= 320)
        hipLaunchKernelGGL((k_rr_chol_rows<5, W>), dim3(1), tb, sh, st, m, gram, hs, L, X, fail, status);
    else
        hipLaunchKernelGGL(k_rr_chol, dim3(1), dim3(kBig), 0, st, m, gram, hs, L, X, fail, status);
}


// 1 / x: hardware reciprocal refined by one Newton step (about 1 ulp);
// used where the result feeds a sign test or an iterative refinement.
__device__ __forceinline__ double rcp1(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// number of eigenvalues of T below x (Sturm sequence of the LDL^T pivots)
__device__ int sturm_count(int m, const double *d, const double *e2, double x, double pivmin)
{
    int c = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
    for (int i = 1; i < m; ++i) {
        q = (d[i] - x) - e2[i - 1] * rcp1(q);
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
    }
    return c;
}

// Gershgorin interval of T, |T| and the pivot floor, from d and e in LDS
// (one wavefront).
struct TriBounds {
    double lo, hi, tnorm, pivmin;
};
__device__ TriBounds tri_bounds(int m, const double *sd, const double *se)
{
    double lo = INFINITY, hi = -INFINITY, emax2 = 0.0;
    for (int i = threadIdx.x; i < m; i += 64) {
        const double r = fabs(se[i]) + (i > 0 ? fabs(se[i - 1]) : 0.0);
        lo = fmin(lo, sd[i] - r);
        hi = fmax(hi, sd[i] + r);
        emax2 = fmax(emax2, se[i] * se[i]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, o));
        hi = fmax(hi, __shfl_xor(hi, o));
        emax2 = fmax(emax2, __shfl_xor(emax2, o));
    }
    TriBounds b;
    b.tnorm = fmax(fabs(lo), fabs(hi));
    b.pivmin = DBL_MIN * fmax(1.0, emax2);
    b.lo = lo - (2.0 * DBL_EPSILON * b.tnorm + 2.0 * b.pivmin);
    b.hi = hi + (2.0 * DBL_EPSILON * b.tnorm + 2.0 * b.pivmin);
    return b;
}

constexpr int kTriMax = 1024;  // largest tridiagonal order of the eigen kernels

// Eigenvalue j of the real symmetric tridiagonal T (d, e), ascending, one
// single-wave work-group per eigenvalue: 64-point multisection of Sturm
// counts, each round shrinking the interval 65-fold, down to an absolute
// width of 2 eps |T| (the accuracy of the eigenvalues of T).
__device__ __forceinline__ void tri_eigvals_body(int bx, int m, const double *__restrict__ d_in,
                                                 const double *__restrict__ e_in, double *__restrict__ lam,
                                                 double *__restrict__ lam2, int nout)
{
    __shared__ double sd[kTriMax], se[kTriMax], se2[kTriMax];
    const int lane = threadIdx.x, j = bx;
    for (int i = lane; i < m; i += 64) {
        sd[i] = d_in[i];
        se[i] = i + 1 < m ? e_in[i] : 0.0;
        se2[i] = se[i] * se[i];
    }
    __syncthreads();
    const TriBounds b = tri_bounds(m, sd, se);
    double a = b.lo, c = b.hi;
    const double target = 2.0 * DBL_EPSILON * b.tnorm + 2.0 * b.pivmin;
    const int rounds = (int)ceil(log(fmax((c - a) / target, 2.0)) / log(65.0)) + 1;
    for (int r = 0; r < rounds; ++r) {
        const double x = a + (c - a) * (double)(lane + 1) / 65.0;
        const unsigned long long above = __ballot(sturm_count(m, sd, se2, x, b.pivmin) > j);
        // eigenvalue j lies in (x_{p-1}, x_p], p = first point above it
        const int p = above ? __builtin_ctzll(above) : 64;
        const double na = p > 0 ? a + (c - a) * (double)p / 65.0 : a;
        const double nc = p < 64 ? a + (c - a) * (double)(p + 1) / 65.0 : c;
        a = na;
        c = nc;
    }
    if (lane == 0) {
        const double v = 0.5 * (a + c);
        lam[j] = v;
        if (lam2 && j < nout) lam2[j] = v;
    }
}
__global__ void __launch_bounds__(64)
k_tri_eigvals(int m, const double *__restrict__ d_in, const double *__restrict__ e_in, double *__restrict__ lam,
              double *__restrict__ lam2, int nout)
{
    tri_eigvals_body(blockIdx.x, m, d_in, e_in, lam, lam2, nout);
}
__global__ void __launch_bounds__(64) k_tri_eigvals_grp(GroupTab t)
{
    int e, bx, by;
    group_block(t, e, bx, by);
    const EigvalsArgs &a = *static_cast<const EigvalsArgs *>(t.args[e]);
    tri_eigvals_body(bx, a.m, a.d, a.e, a.lam, a.lam2, a.nout);
}


// Eigenvectors of T by inverse iteration, one single-wave work-group per
// cluster of eigenvalues (gaps below 1e-5 |T|; most clusters have one
// member), started by the work-group of its first member.  Per member: LU
// with partial pivoting of T - s I (s at least 10 eps |T| above the
// previous member's), three solves from a fixed start vector, members after
// the first orthogonalised against the earlier ones (modified Gram-Schmidt)
// after every solve.  The LU factors and the iterate live in LDS; lane 0
// runs the serial recurrences, the wavefront the vector operations.
// Z: column j (m doubles) of eigenvector j.
__device__ __forceinline__ void tri_eigvecs_body(int bx, int m, const double *__restrict__ d_in,
                                                 const double *__restrict__ e_in, const double *__restrict__ lam,
                                                 double *__restrict__ Z)
{
    extern __shared__ double lds[];
    double *sd = lds, *se = lds + m;
    double *S0 = lds + 2 * m, *S1 = lds + 3 * m, *S2 = lds + 4 * m, *S3 = lds + 5 * m, *PV = lds + 6 * m;
    double *zw = lds + 7 * m;
    __shared__ double s_scale;
    const int lane = threadIdx.x, j0 = bx;
    for (int i = lane; i < m; i += 64) {
        sd[i] = d_in[i];
        se[i] = i + 1 < m ? e_in[i] : 0.0;
    }
    __syncthreads();
    const TriBounds b = tri_bounds(m, sd, se);
    const double ortol = 1e-5 * b.tnorm, pert = 10.0 * DBL_EPSILON * b.tnorm;
    if (j0 > 0 && lam[j0] - lam[j0 - 1] <= ortol) return;  // not a cluster start
    int cend = j0 + 1;
    while (cend < m && lam[cend] - lam[cend - 1] <= ortol) ++cend;
    const double tiny = DBL_EPSILON * b.tnorm + DBL_MIN;
    double prev_shift = 0.0;
    for (int j = j0; j < cend; ++j) {
        double s = lam[j];
        if (j > j0 && s - prev_shift < pert) s = prev_shift + pert;
        prev_shift = s;
        if (lane == 0) {
            // S0 multipliers, S1 reciprocal pivots, S2 / S3 first / second
            // superdiagonal of U, PV = 1 where rows k and k+1 were swapped
            double dk = sd[0] - s, uk = se[0];
            for (int k = 0; k + 1 < m; ++k) {
                const double lk = se[k];
                const double dn = sd[k + 1] - s, un = se[k + 1];
                if (fabs(dk) >= fabs(lk)) {
                    const double r = rcp1(dk == 0.0 ? tiny : dk);
                    const double f = lk * r;
                    S0[k] = f;
                    S1[k] = r;
                    S2[k] = uk;
                    S3[k] = 0.0;
                    PV[k] = 0.0;
                    dk = fma(-f, uk, dn);
                    uk = un;
                } else {
                    const double f = dk * rcp1(lk);
                    S0[k] = f;
                    S1[k] = rcp1(lk);
                    S2[k] = dn;
                    S3[k] = un;
                    PV[k] = 1.0;
                    dk = fma(-f, dn, uk);
                    uk = -f * un;
                }
            }
            S1[m - 1] = rcp1(dk == 0.0 ? tiny : dk);
            S2[m - 1] = 0.0;
            S3[m - 1] = 0.0;
        }
        // start vector: fixed pseudo-random entries in [0.5, 1.5)
        for (int k = lane; k < m; k += 64) {
            unsigned h = (unsigned)(k + 1) * 2654435761u ^ (unsigned)(j + 7) * 40503u;
            h ^= h >> 13;
            h *= 0x5bd1e995u;
            h ^= h >> 15;
            zw[k] = 0.5 + (double)(h & 0xffffff) / 16777216.0;
        }
        __syncthreads();
        for (int it = 0; it < 3; ++it) {
            if (lane == 0) {
                // forward: row swaps and multipliers; zc = running z[k]
                double zc = zw[0];
                for (int k = 0; k + 1 < m; ++k) {
                    const double zn = zw[k + 1], f = S0[k];
                    if (PV[k] != 0.0) {
                        zw[k] = zn;
                        zc = fma(-f, zn, zc);
                    } else {
                        zw[k] = zc;
                        zc = fma(-f, zc, zn);
                    }
                }
                // back substitution with U
                double z1 = zc * S1[m - 1], z2 = 0.0, n2 = z1 * z1;
                zw[m - 1] = z1;
                for (int k = m - 2; k >= 0; --k) {
                    const double v = (zw[k] - S2[k] * z1 - S3[k] * z2) * S1[k];
                    zw[k] = v;
                    n2 = fma(v, v, n2);
                    z2 = z1;
                    z1 = v;
                }
                s_scale = n2 > 0.0 ? 1.0 / sqrt(n2) : 1.0;
            }
            __syncthreads();
            const double sc = s_scale;
            for (int k = lane; k < m; k += 64) zw[k] *= sc;
            if (j > j0) {
                __syncthreads();
                for (int p = j0; p < j; ++p) {
                    const double *__restrict__ zp = Z + (int64_t)p * m;
                    double dot = 0.0;
                    for (int k = lane; k < m; k += 64) dot += zp[k] * zw[k];
                    for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o);
                    for (int k = lane; k < m; k += 64) zw[k] -= dot * zp[k];
                }
                double q2 = 0.0;
                for (int k = lane; k < m; k += 64) q2 += zw[k] * zw[k];
                for (int o = 32; o > 0; o >>= 1) q2 += __shfl_xor(q2, o);
                const double sq = q2 > 0.0 ? 1.0 / sqrt(q2) : 1.0;
                for (int k = lane; k < m; k += 64) zw[k] *= sq;
            }
            __syncthreads();
        }
        double *__restrict__ z = Z + (int64_t)j * m;
        for (int k = lane; k < m; k += 64) z[k] = zw[k];
        __threadfence_block();
        __syncthreads();
    }
}
__global__ void __launch_bounds__(64)
k_tri_eigvecs(int m, const double *__restrict__ d_in, const double *__restrict__ e_in, const double *__restrict__ lam,
              double *__restrict__ Z)
{
    tri_eigvecs_body(blockIdx.x, m, d_in, e_in, lam, Z);
}
__global__ void __launch_bounds__(64) k_tri_eigvecs_grp(GroupTab t)
{
    int e, bx, by;
    group_block(t, e, bx, by);
    const EigvecsArgs &a = *static_cast<const EigvecsArgs *>(t.args[e]);
    tri_eigvecs_body(bx, a.m, a.d, a.e, a.lam, a.Z);
}


// Y = Q Z (complex m x m from real Z), one column per single-wave block:
// y <- H_k y = y - tau_k v_k (v_k^H y), k = m-2 .. 0.
__device__ __forceinline__ void backtransform_body(int bx, int m, const double2 *__restrict__ A,
                                                   const double2 *__restrict__ tau, const double *__restrict__ Z,
                                                   double2 *__restrict__ Y)
{
    extern __shared__ double2 y[];
    const int j = bx, lane = threadIdx.x;
    for (int i = lane; i < m; i += 64) y[i] = make_double2(Z[(int64_t)j * m + i], 0.0);
    __syncthreads();
    for (int k = m - 2; k >= 0; --k) {
        const double2 tk = tau[k];
        if (tk.x == 0.0 && tk.y == 0.0) continue;
        const int n = m - k - 1;
        const double2 *v = A + (int64_t)k * m + k + 1;
        double sr = 0.0, si = 0.0;
        for (int i = lane; i < n; i += 64) {
            const double2 t = cjmul(v[i], y[k + 1 + i]);
            sr += t.x;
            si += t.y;
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        sr = __shfl(sr, 0, 64);
        si = __shfl(si, 0, 64);
        const double2 f = cmul_(tk, make_double2(sr, si));
        __syncthreads();
        for (int i = lane; i < n; i += 64) {
            const double2 t = cmul_(v[i], f);
            y[k + 1 + i] = make_double2(y[k + 1 + i].x - t.x, y[k + 1 + i].y - t.y);
        }
        __syncthreads();
    }
    for (int i = lane; i < m; i += 64) Y[(int64_t)j * m + i] = y[i];
}
__global__ void __launch_bounds__(64)
k_backtransform(int m, const double2 *__restrict__ A, const double2 *__restrict__ tau, const double *__restrict__ Z,
                double2 *__restrict__ Y)
{
    backtransform_body(blockIdx.x, m, A, tau, Z, Y);
}
__global__ void __launch_bounds__(64) k_backtransform_grp(GroupTab t)
{
    int e, bx, by;
    group_block(t, e, bx, by);
    const BacktArgs &a = *static_cast<const BacktArgs *>(t.args[e]);
    backtransform_body(bx, a.m, a.A, a.tau, a.Z, a.Y);
}


// M = L^H diag(dk) L (projector part of the shift bound)
__global__ void k_lhdl(int m, const double2 *__restrict__ L, const double *__restrict__ dk, double2 *__restrict__ M)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= m) return;
    double2 acc = make_double2(0.0, 0.0);
    for (int k = 0; k < m; ++k) {
        const double2 t = cjmul(L[(int64_t)i * m + k], L[(int64_t)j * m + k]);
        acc.x += dk[k] * t.x;
        acc.y += dk[k] * t.y;
    }
    M[(int64_t)j * m + i] = acc;
}

__global__ void __launch_bounds__(256) k_vmin(int64_t n, const double *__restrict__ v, double *__restrict__ out)
{
    __shared__ double red[4];
    double mn = INFINITY;
    for (int64_t i = threadIdx.x; i < n; i += 256) mn = fmin(mn, v[i]);
    mn = -block_max<256>(-mn, red);
    if (threadIdx.x == 0) out[0] = mn;
}

__global__ void k_shift_final(const double *__restrict__ vmin, const double *__restrict__ lam, int has_nl,
                              const int32_t *__restrict__ fail, double *__restrict__ sigma)
{
    double l = has_nl ? lam[0] : 0.0;
    if (has_nl && fail[0]) l = NAN;
    sigma[0] = vmin[0] + (l < 0.0 ? l : 0.0) - 0.1;
    if (l != l) sigma[0] = NAN;
}

// After an outer iteration: stats row, next shift, convergence flag.
__device__ __forceinline__ void bookkeep_body(int nb, int n_conv, int shift_mode, double sigma_lb, double tol_res,
                                              const double *__restrict__ eps, const double *__restrict__ res,
                                              double *__restrict__ sig_all, double *__restrict__ sig_out,
                                              double *__restrict__ stats_row, int32_t *__restrict__ conv)
{
    double sigma = sigma_lb;
    if (shift_mode == PARO_SHIFT_ADAPTIVE && res[0] < 0.1) {
        const double s = eps[0] - 0.05 - res[0];
        if (s > sigma) sigma = s;
    }
    double rmax = 0.0;
    for (int b = 0; b < n_conv; ++b) rmax = fmax(rmax, res[b]);
    const int ok = tol_res > 0.0 && rmax <= tol_res;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) sig_all[b] = sigma;
    if (threadIdx.x == 0) {
        sig_out[0] = sigma;
        conv[0] = ok;
    }
    if (stats_row) {
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
            stats_row[b] = eps[b];
            stats_row[nb + b] = res[b];
        }
        if (threadIdx.x == 0) {
            stats_row[2 * nb] = sigma;
            stats_row[2 * nb + 1] = ok ? 1.0 : 0.0;
        }
    }
}
__global__ void k_bookkeep(int nb, int n_conv, int shift_mode, double sigma_lb, double tol_res,
                           const double *__restrict__ eps, const double *__restrict__ res, double *__restrict__ sig_all,
                           double *__restrict__ sig_out, double *__restrict__ stats_row, int32_t *__restrict__ conv)
{
    bookkeep_body(nb, n_conv, shift_mode, sigma_lb, tol_res, eps, res, sig_all, sig_out, stats_row, conv);
}
// one work-group per entry; it: the outer iteration whose statistics row is written
__global__ void k_bookkeep_grp(GroupTab t, int it)
{
    const BookArgs &a = *static_cast<const BookArgs *>(t.args[blockIdx.x]);
    bookkeep_body(a.nb, a.n_conv, a.shift_mode, a.sigma_lb, a.tol_res, a.eps, a.res, a.sig_all, a.sig_out,
                  a.stats ? a.stats + (size_t)(it + 1) * a.row : nullptr, a.conv);
}


}  // namespace

// dreal layout: d[m] e[m] tau[2m] lam[m] vmin[1] fail(int)[2] | Z[m*m]
struct DenseScratch {
    double *d, *e, *lam, *vmin;
    double2 *tau;
    int32_t *fail;
    double *Z;
    // exchange buffers of the multi-work-group tridiagonalisation:
    // v (2 x (m + 1)), partial y (2 x G x m, G up to kTriDistG2), flags (2 m + 1 int32)
    double2 *vbuf, *ypart;
    int32_t *flags;
};

static DenseScratch dense_scratch(const Workspace &w, int m)
{
    DenseScratch s;
    double *p = w.dreal;
    s.d = p;
    s.e = p + m;
    s.tau = reinterpret_cast<double2 *>(p + 2 * m);
    s.lam = p + 4 * m;
    s.vmin = p + 5 * m;
    s.fail = reinterpret_cast<int32_t *>(p + 5 * m + 1);
    s.Z = p + 5 * m + 2;
    size_t off = 5 * (size_t)m + 2 + (size_t)m * m;
    off += off & 1;  // 16-byte alignment of the complex buffers
    s.vbuf = reinterpret_cast<double2 *>(p + off);
    s.ypart = s.vbuf + 2 * ((size_t)m + 1);
    s.flags = reinterpret_cast<int32_t *>(s.ypart + 2 * (size_t)kTriDistG2 * m);
    return s;
}

size_t dense_real_elems(int mmax)
{
    const size_t m = mmax;
    return 5 * m + 2 + m * m + 1 + 2 * (2 * (m + 1) + 2 * (size_t)kTriDistG2 * m) + (2 * m + 2) / 2 + 1;
}

// The distributed tridiagonalisation (ordinary launch of G work-groups),
// one size class; false when the device cannot hold them (the caller then
// uses a one-work-group variant).
template <int G, int NT, int MMAX>
static bool launch_tridiag_dist_g(hipStream_t st, int m, double2 *Hh, const DenseScratch &s, int32_t *status)
{
    const void *k = reinterpret_cast<const void *>(k_tridiag_dist<G, NT>);
    static const bool ok = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)tridiag_dist_lds_bytes<G>(MMAX)) == hipSuccess &&
                           dist_grid_fits(k, G, NT, tridiag_dist_lds_bytes<G>(MMAX));
    if (!ok) return false;
    hipLaunchKernelGGL(k_fill_i32, dim3((2 * m + 1 + 255) / 256), dim3(256), 0, st, 2 * m + 1, s.flags, 0);
    hipLaunchKernelGGL((k_tridiag_dist<G, NT>), dim3(G), dim3(NT), tridiag_dist_lds_bytes<G>(m), st, m, Hh, s.d,
                       s.e, s.tau, s.vbuf, s.ypart, s.flags, status);
    return true;
}

static bool launch_tridiag_dist(hipStream_t st, int m, double2 *Hh, const DenseScratch &s, int32_t *status)
{
    if (m >= kTriDistMinTridiag && m <= kTriDistMax)
        return launch_tridiag_dist_g<kTriDistG, kTriDistThreads, kTriDistMax>(st, m, Hh, s, status);
    if (m > kTriDistMax && m <= kTriDistMax2)
        return launch_tridiag_dist_g<kTriDistG2, kTriDistThreads2, kTriDistMax2>(st, m, Hh, s, status);
    return false;
}

static hipError_t eig_pipeline(hipStream_t st, int m, double2 *Hh, const DenseScratch &s, double *eps_out,
                               int nout, double2 *Yout, bool vectors, int32_t *status = nullptr)
{
    static const hipError_t lds_attr = hipFuncSetAttribute(
        reinterpret_cast<const void *>(k_tridiag_rows<2, true, kTriWavesLds>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)tridiag_lds_bytes(kTridiagLdsMax, true));
    static const hipError_t reg_attr = hipFuncSetAttribute(reinterpret_cast<const void *>(k_tridiag_reg),
                                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTriRegLds);
    const dim3 tl(64 * kTriWavesLds), tg(64 * kTriWavesGlobal);
    const size_t gb = tridiag_lds_bytes(m, false);
    if (m <= kTridiagLdsMax && lds_attr == hipSuccess)
        hipLaunchKernelGGL((k_tridiag_rows<2, true, kTriWavesLds>), dim3(1), tl, tridiag_lds_bytes(m, true), st, m,
                           Hh, s.d, s.e, s.tau);
    else if (m >= kTriRegMin && m <= kTriRegMax && reg_attr == hipSuccess)
        hipLaunchKernelGGL(k_tridiag_reg, dim3(1), dim3(64 * kTriRegWaves), kTriRegLds, st, m, Hh, s.d, s.e, s.tau);
    else if (launch_tridiag_dist(st, m, Hh, s, status)) {
    } else if (m <= 128)
        hipLaunchKernelGGL((k_tridiag_rows<2, false, kTriWavesGlobal>), dim3(1), tg, gb, st, m, Hh, s.d, s.e, s.tau);
    else if (m <= 192)
        hipLaunchKernelGGL((k_tridiag_rows<3, false, kTriWavesGlobal>), dim3(1), tg, gb, st, m, Hh, s.d, s.e, s.tau);
    else if (m <= 256)
        hipLaunchKernelGGL((k_tridiag_rows<4, false, kTriWavesGlobal>), dim3(1), tg, gb, st, m, Hh, s.d, s.e, s.tau);
    else if (m <= 64 * kTridiagRowsMax)
        hipLaunchKernelGGL((k_tridiag_rows<kTridiagRowsMax, false, kTriWavesGlobal>), dim3(1), tg, gb, st, m, Hh, s.d,
                           s.e, s.tau);
    else
        hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(kBig), 0, st, m, Hh, s.d, s.e, s.tau);
    hipLaunchKernelGGL(k_tri_eigvals, dim3(m), dim3(64), 0, st, m, s.d, s.e, s.lam, eps_out, nout);
    if (vectors)
        hipLaunchKernelGGL(k_tri_eigvecs, dim3(m), dim3(64), 8 * (size_t)m * sizeof(double), st, m, s.d, s.e, s.lam,
                           s.Z);
    if (vectors)
        hipLaunchKernelGGL(k_backtransform, dim3(m), dim3(64), (size_t)m * sizeof(double2), st, m, Hh, s.tau, s.Z,
                           Yout);
    return hipGetLastError();
}

hipError_t launch_rr_dense(const Plan &pl, const Workspace &w, int m, int n_keep, double *eps_out, double2 *C)
{
    if (m > kBig) return hipErrorInvalidValue;
    hipStream_t st = pl.stream;
    DenseScratch s = dense_scratch(w, m);
    double2 *L = w.dense[0], *X = w.dense[1], *Hh = w.dense[2], *Y = w.dense[3];
    const size_t colshm = (size_t)m * sizeof(double2);
    launch_chol(st, m, w.gram, 1, L, X, s.fail, pl.status, s.flags);
    // X <- L^-1 Hs;  Hh <- L^-1 X^H = L^-1 Hs L^-H
    hipLaunchKernelGGL(k_trsm_col, dim3(m), dim3(64), colshm, st, m, L, X, 0, 0, X);
    hipLaunchKernelGGL(k_trsm_col, dim3(m), dim3(64), colshm, st, m, L, X, 1, 0, Hh);
    hipError_t e = eig_pipeline(st, m, Hh, s, eps_out, n_keep, Y, true, pl.status);
    if (e != hipSuccess) return e;
    // C = L^-H Y
    hipLaunchKernelGGL(k_trsm_col, dim3(m), dim3(64), colshm, st, m, L, Y, 0, 1, C);
    return hipGetLastError();
}

// Standalone Hermitian eigensolver on the device (the Rayleigh-Ritz
// eigensolve without the overlap): A (m x m, column-major) is copied to
// dense[2]; eigenvalues to w (ascending), eigenvectors to V.
hipError_t launch_heev(hipStream_t st, const Workspace &w, int m, const double2 *A, double *wout, double2 *V)
{
    if (m > kBig) return hipErrorInvalidValue;
    DenseScratch s = dense_scratch(w, m);
    hipError_t e = hipMemcpyAsync(w.dense[2], A, sizeof(double2) * m * m, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    return eig_pipeline(st, m, w.dense[2], s, wout, m, V, true);
}

hipError_t launch_shift_bound(const Plan &pl, const Workspace &w, double *sigma)
{
    hipStream_t st = pl.stream;
    const int np = pl.nproj;
    DenseScratch s = dense_scratch(w, np > 0 ? np : 1);
    const int64_t nv = (int64_t)pl.grid[0] * pl.grid[1] * pl.grid[2];
    hipLaunchKernelGGL(k_vmin, dim3(1), dim3(256), 0, st, nv, pl.vplane, s.vmin);
    if (np > 0) {
        // G = B^H B, Cholesky, M = L^H D L, lowest eigenvalue
        hipError_t err = gemm_hn(st, np, np, pl.ng, pl.beta, pl.ldv, pl.beta, pl.ldv, w.gram, np, w.part,
                                 w.part_elems, nullptr, nullptr);
        if (err != hipSuccess) return err;
        launch_chol(st, np, w.gram, 0, w.dense[0], w.dense[1], s.fail, pl.status);
        hipLaunchKernelGGL(k_lhdl, dim3((np + 63) / 64, np), dim3(64), 0, st, np, w.dense[0], pl.dkb, w.dense[2]);
        err = eig_pipeline(st, np, w.dense[2], s, nullptr, 0, nullptr, false);
        if (err != hipSuccess) return err;
    }
    hipLaunchKernelGGL(k_shift_final, dim3(1), dim3(1), 0, st, s.vmin, s.lam, np > 0 ? 1 : 0, s.fail, sigma);
    return hipGetLastError();
}

hipError_t launch_bookkeeping(const Plan &pl, int nb, const paro_iter_opts &o, const double *eps, const double *res,
                              double *sig_all, double *sig_out, double *stats_row, int32_t *conv)
{
    const int nconv = o.n_conv > 0 && o.n_conv <= nb ? o.n_conv : nb;
    hipLaunchKernelGGL(k_bookkeep, dim3(1), dim3(256), 0, pl.stream, nb, nconv, o.shift_mode, o.sigma_lb, o.tol_res,
                       eps, res, sig_all, sig_out, stats_row, conv);
    return hipGetLastError();
}

}  // namespace paro

namespace paro {

// ---------------------------------------------------------------- grouped launches
// The dense part of Rayleigh-Ritz (launch_rr_dense) for many cells at once,
// for m <= 92: the one-work-group Cholesky, the three triangular solves,
// the LDS-resident tridiagonalisation, eigenvalues, eigenvectors and the
// back-transformation, each one launch for all cells.
bool rr_dense_groupable(int m) { return m >= 1 && m <= kTridiagLdsMax; }

void describe_rr_dense(const Plan &pl, const Workspace &w, int m, int n_keep, double *eps_out, double2 *C,
                       GroupFinishArgs &f)
{
    DenseScratch s = dense_scratch(w, m);
    double2 *L = w.dense[0], *X = w.dense[1], *Hh = w.dense[2], *Y = w.dense[3];
    f.chol = CholArgs{w.gram, L, X, s.fail, pl.status, m, 1};
    f.trsm[0] = TrsmArgs{L, X, X, m, 0, 0};
    f.trsm[1] = TrsmArgs{L, X, Hh, m, 1, 0};
    f.trsm[2] = TrsmArgs{L, Y, C, m, 0, 1};
    f.tri = TridiagArgs{Hh, s.d, s.e, s.tau, m};
    f.evals = EigvalsArgs{s.d, s.e, s.lam, eps_out, m, n_keep};
    f.evecs = EigvecsArgs{s.d, s.e, s.lam, s.Z, m};
    f.back = BacktArgs{Hh, s.tau, s.Z, Y, m};
}

void describe_bookkeeping(const Plan &pl, int nb, const paro_iter_opts &o, const double *eps, const double *res,
                          double *sig_all, double *sig_out, double *stats, int32_t *conv, GroupFinishArgs &f)
{
    (void)pl;
    const int nconv = o.n_conv > 0 && o.n_conv <= nb ? o.n_conv : nb;
    f.book = BookArgs{eps, res, sig_all, sig_out, stats, conv, o.sigma_lb, o.tol_res, nb, nconv, o.shift_mode,
                      2 * nb + 2};
}

namespace {

// one entry per cell, blocks per entry from blocks_of(cell); launches every kGroupMax entries
template <class A, class B, class L>
void group_dense(const GroupCell *cells, int n, A args_of, B blocks_of, L launch)
{
    GroupBuilder g;
    int mmax = 0;
    for (int i = 0; i < n; ++i) {
        const int m = cells[i].host->fin.chol.m;
        const int64_t nbk = blocks_of(m);
        g.add(args_of(cells[i].dev), nbk, (int)nbk);
        mmax = std::max(mmax, m);
        if (g.full() || i == n - 1) {
            launch(g, mmax);
            g = GroupBuilder();
            mmax = 0;
        }
    }
}

}  // namespace

hipError_t launch_rr_dense_grouped(hipStream_t s, const GroupCell *cells, int n)
{
    if (n <= 0) return hipSuccess;
    static const hipError_t lds_attr = hipFuncSetAttribute(
        reinterpret_cast<const void *>(k_tridiag_rows_grp<2, true, kTriWavesLds>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)tridiag_lds_bytes(kTridiagLdsMax, true));
    if (lds_attr != hipSuccess) return lds_attr;
    constexpr int W = 16;
    auto one = [](int) { return (int64_t)1; };
    auto cols = [](int m) { return (int64_t)m; };
    group_dense(cells, n, [](const GroupCellDesc *d) { return (const void *)&d->fin.chol; }, one,
                [&](const GroupBuilder &g, int mmax) {
                    hipLaunchKernelGGL((k_rr_chol_rows_grp<2, W>), dim3(g.t.n), dim3(64 * W),
                                       sizeof(double2) * (size_t)mmax, s, g.t);
                });
    for (int k = 0; k < 2; ++k)
        group_dense(cells, n, [k](const GroupCellDesc *d) { return (const void *)&d->fin.trsm[k]; }, cols,
                    [&](const GroupBuilder &g, int mmax) {
                        hipLaunchKernelGGL(k_trsm_col_grp, dim3((unsigned)g.total), dim3(64),
                                           sizeof(double2) * (size_t)mmax, s, g.t);
                    });
    group_dense(cells, n, [](const GroupCellDesc *d) { return (const void *)&d->fin.tri; }, one,
                [&](const GroupBuilder &g, int mmax) {
                    hipLaunchKernelGGL((k_tridiag_rows_grp<2, true, kTriWavesLds>), dim3(g.t.n),
                                       dim3(64 * kTriWavesLds), tridiag_lds_bytes(mmax, true), s, g.t);
                });
    group_dense(cells, n, [](const GroupCellDesc *d) { return (const void *)&d->fin.evals; }, cols,
                [&](const GroupBuilder &g, int) {
                    hipLaunchKernelGGL(k_tri_eigvals_grp, dim3((unsigned)g.total), dim3(64), 0, s, g.t);
                });
    group_dense(cells, n, [](const GroupCellDesc *d) { return (const void *)&d->fin.evecs; }, cols,
                [&](const GroupBuilder &g, int mmax) {
                    hipLaunchKernelGGL(k_tri_eigvecs_grp, dim3((unsigned)g.total), dim3(64),
                                       8 * (size_t)mmax * sizeof(double), s, g.t);
                });
    group_dense(cells, n, [](const GroupCellDesc *d) { return (const void *)&d->fin.back; }, cols,
                [&](const GroupBuilder &g, int mmax) {
                    hipLaunchKernelGGL(k_backtransform_grp, dim3((unsigned)g.total), dim3(64),
                                       sizeof(double2) * (size_t)mmax, s, g.t);
                });
    group_dense(cells, n, [](const GroupCellDesc *d) { return (const void *)&d->fin.trsm[2]; }, cols,
                [&](const GroupBuilder &g, int mmax) {
                    hipLaunchKernelGGL(k_trsm_col_grp, dim3((unsigned)g.total), dim3(64),
                                       sizeof(double2) * (size_t)mmax, s, g.t);
                });
    return hipGetLastError();
}

hipError_t launch_bookkeeping_grouped(hipStream_t s, const GroupCell *cells, int n, int it)
{
    GroupBuilder g;
    for (int i = 0; i < n; ++i) {
        g.add(&cells[i].dev->fin.book, 1, 1);
        if (g.full() || i == n - 1) {
            hipLaunchKernelGGL(k_bookkeep_grp, dim3(g.t.n), dim3(256), 0, s, g.t, it);
            g = GroupBuilder();
        }
    }
    return hipGetLastError();
}

}  // namespace paro
