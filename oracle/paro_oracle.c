/*
 * Plain CPU oracle for the ParO plane-wave eigensolver hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code with the GPU library and is written for readability, not speed.
 *
 * Paper: Pan, Dai, de Gironcoli, Gong, Rignanese, Zhou, "A parallel
 * orbital-updating based plane-wave basis method for electronic structure
 * calculations" (arXiv 1702.04045).  Every function cites the passage it
 * follows.  Readings of passages where the paper is silent or garbled:
 *   - matrix elements of the local potential use G_m - G_n (the printed
 *     G_m + G_n would not give a Hermitian matrix);
 *   - the inner product is the Hermitian one (c^H d);
 *   - the integral over the cell is the grid quadrature of V sampled on the
 *     FFT grid: Vt(k) = (1/N) sum_j V_j exp(-2 pi i k.j/N);
 *   - the source problem of Algorithm 1 step 3 is solved with a shift,
 *     (H - sigma) u = (eps - sigma) psi, by Teter-preconditioned CG started
 *     from u = psi (sigma = 0 is the printed equation);
 *   - KB projectors are Gaussian s and p functions normalised on the sphere.
 *
 * All floating point is IEEE double; complex numbers are C99 double complex.
 * Orbital blocks are band-major: coefficient g of band b at [b*ng + g].
 * Small dense m x m matrices are column-major: entry (i,j) at [i + j*m].
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORC_F_NEGCURV 1
#define ORC_F_CHOL 2
#define ORC_F_NAN 4

static const double TWO_PI = 6.283185307179586476925286766559;

/* ------------------------------------------------------------------ */
/* Reciprocal lattice: b_i . a_j = 2 pi delta_ij (Section 2.2, G such   */
/* that exp(iG.R) = 1 for every lattice vector R).                      */
/* cell rows are a1, a2, a3; output rows are b1, b2, b3.                */
/* ------------------------------------------------------------------ */
static double recip(const double a[9], double b[9])
{
    double c[9];
    c[0] = a[4] * a[8] - a[5] * a[7];
    c[1] = a[5] * a[6] - a[3] * a[8];
    c[2] = a[3] * a[7] - a[4] * a[6];
    c[3] = a[7] * a[2] - a[8] * a[1];
    c[4] = a[8] * a[0] - a[6] * a[2];
    c[5] = a[6] * a[1] - a[7] * a[0];
    c[6] = a[1] * a[5] - a[2] * a[4];
    c[7] = a[2] * a[3] - a[0] * a[5];
    c[8] = a[0] * a[4] - a[1] * a[3];
    double det = a[0] * c[0] + a[1] * c[1] + a[2] * c[2];
    /* b1 = 2pi (a2 x a3)/det, b2 = 2pi (a3 x a1)/det, b3 = 2pi (a1 x a2)/det */
    for (int i = 0; i < 9; ++i) b[i] = TWO_PI * c[i] / det;
    return fabs(det);
}

static void gvec_of(const double b[9], int n1, int n2, int n3, double g[3])
{
    for (int d = 0; d < 3; ++d) g[d] = n1 * b[d] + n2 * b[3 + d] + n3 * b[6 + d];
}

/* ------------------------------------------------------------------ */
/* G-sphere, cutoff condition (e3): (1/2)|G|^2 <= E_cut at k = 0.       */
/* Enumerated in lexicographic order of the Miller indices (n1,n2,n3).  */
/* Boundary ties are included up to a relative 1e-12.                   */
/* Returns the number of points; fills miller (n x 3) if non-NULL.      */
/* ------------------------------------------------------------------ */
int64_t orc_sphere(const double *cell, double ecut, int32_t *miller,
                   int64_t cap, int32_t *nmax_out)
{
    double b[9];
    recip(cell, b);
    double gmax = sqrt(2.0 * ecut);
    int box[3];
    for (int d = 0; d < 3; ++d) {
        double alen = sqrt(cell[3 * d] * cell[3 * d] + cell[3 * d + 1] * cell[3 * d + 1] +
                           cell[3 * d + 2] * cell[3 * d + 2]);
        box[d] = (int)floor(gmax * alen / TWO_PI) + 1; /* |n_d| = |G.a_d|/2pi */
    }
    int64_t n = 0;
    int nm[3] = {0, 0, 0};
    for (int n1 = -box[0]; n1 <= box[0]; ++n1)
        for (int n2 = -box[1]; n2 <= box[1]; ++n2)
            for (int n3 = -box[2]; n3 <= box[2]; ++n3) {
                double g[3];
                gvec_of(b, n1, n2, n3, g);
                double kin = 0.5 * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
                if (kin <= ecut * (1.0 + 1e-12)) {
                    if (miller && n < cap) {
                        miller[3 * n] = n1;
                        miller[3 * n + 1] = n2;
                        miller[3 * n + 2] = n3;
                    }
                    ++n;
                    if (abs(n1) > nm[0]) nm[0] = abs(n1);
                    if (abs(n2) > nm[1]) nm[1] = abs(n2);
                    if (abs(n3) > nm[2]) nm[2] = abs(n3);
                }
            }
    if (nmax_out) for (int d = 0; d < 3; ++d) nmax_out[d] = nm[d];
    return n;
}

/* ------------------------------------------------------------------ */
/* Radix-2 FFT (iterative Cooley-Tukey, bit reversal first).            */
/* x_k <- sum_j x_j exp(sign * 2 pi i j k / n), unnormalised.           */
/* tw holds exp(sign * 2 pi i j / n) for j < n/2.                       */
/* ------------------------------------------------------------------ */
static void twiddles(int n, int sign, cplx *tw)
{
    for (int j = 0; j < n / 2; ++j) {
        double ang = TWO_PI * (double)j / (double)n;
        tw[j] = cos(ang) + (double)sign * sin(ang) * I;
    }
}

static void fft_line(cplx *x, int n, const cplx *tw)
{
    if (n <= 1) return;
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cplx t = x[i]; x[i] = x[j]; x[j] = t; }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len >> 1, step = n / len;
        for (int k = 0; k < half; ++k) {
            cplx w = tw[k * step];
            for (int s = 0; s < n; s += len) {
                cplx a = x[s + k];
                cplx bb = x[s + k + half] * w;
                x[s + k] = a + bb;
                x[s + k + half] = a - bb;
            }
        }
    }
}

void orc_fft1d(cplx *x, int32_t n, int32_t sign)
{
    if (n <= 0 || (n & (n - 1))) return; /* radix 2 only */
    cplx *tw = (cplx *)malloc(sizeof(cplx) * (n / 2 + 1));
    twiddles(n, sign, tw);
    fft_line(x, n, tw);
    free(tw);
}

/* 3-D transform of an M1 x M2 x M3 C-order array, one axis at a time. */
void orc_fft3d(cplx *x, const int32_t *M, int32_t sign)
{
    int m1 = M[0], m2 = M[1], m3 = M[2];
    int mx = m1 > m2 ? m1 : m2;
    if (m3 > mx) mx = m3;
    cplx *line = (cplx *)malloc(sizeof(cplx) * mx);
    cplx *tw1 = (cplx *)malloc(sizeof(cplx) * (m1 / 2 + 1));
    cplx *tw2 = (cplx *)malloc(sizeof(cplx) * (m2 / 2 + 1));
    cplx *tw3 = (cplx *)malloc(sizeof(cplx) * (m3 / 2 + 1));
    twiddles(m1, sign, tw1);
    twiddles(m2, sign, tw2);
    twiddles(m3, sign, tw3);
    for (int i = 0; i < m1 * m2; ++i) fft_line(x + (int64_t)i * m3, m3, tw3);
    for (int i1 = 0; i1 < m1; ++i1)
        for (int i3 = 0; i3 < m3; ++i3) {
            for (int i2 = 0; i2 < m2; ++i2) line[i2] = x[((int64_t)i1 * m2 + i2) * m3 + i3];
            fft_line(line, m2, tw2);
            for (int i2 = 0; i2 < m2; ++i2) x[((int64_t)i1 * m2 + i2) * m3 + i3] = line[i2];
        }
    for (int i2 = 0; i2 < m2; ++i2)
        for (int i3 = 0; i3 < m3; ++i3) {
            for (int i1 = 0; i1 < m1; ++i1) line[i1] = x[((int64_t)i1 * m2 + i2) * m3 + i3];
            fft_line(line, m1, tw1);
            for (int i1 = 0; i1 < m1; ++i1) x[((int64_t)i1 * m2 + i2) * m3 + i3] = line[i1];
        }
    free(line); free(tw1); free(tw2); free(tw3);
}

/* ------------------------------------------------------------------ */
/* Fourier coefficients of the local potential by a direct DFT on the   */
/* native grid (the integral of the matrix element in (e5), as a grid   */
/* quadrature): Vt(k) = (1/N) sum_j V_j exp(-2 pi i sum_d k_d j_d/N_d)  */
/* for |k_d| <= K_d.  Output C order [k1+K1][k2+K2][k3+K3].             */
/* ------------------------------------------------------------------ */
static cplx phase(int64_t kj, int n)
{
    int64_t r = kj % n;
    if (r < 0) r += n;
    double ang = TWO_PI * (double)r / (double)n;
    return cos(ang) - sin(ang) * I;
}

void orc_vtilde(const int32_t *grid, const double *v, const int32_t *K, cplx *out)
{
    int n1 = grid[0], n2 = grid[1], n3 = grid[2];
    int k1n = 2 * K[0] + 1, k2n = 2 * K[1] + 1, k3n = 2 * K[2] + 1;
    cplx *t1 = (cplx *)malloc(sizeof(cplx) * (size_t)n1 * n2 * k3n);
    cplx *t2 = (cplx *)malloc(sizeof(cplx) * (size_t)n1 * k2n * k3n);
    /* sum over j3 */
    for (int j1 = 0; j1 < n1; ++j1)
        for (int j2 = 0; j2 < n2; ++j2)
            for (int a = 0; a < k3n; ++a) {
                int k3 = a - K[2];
                cplx s = 0;
                for (int j3 = 0; j3 < n3; ++j3)
                    s += v[((int64_t)j1 * n2 + j2) * n3 + j3] * phase((int64_t)k3 * j3, n3);
                t1[((int64_t)j1 * n2 + j2) * k3n + a] = s;
            }
    /* sum over j2 */
    for (int j1 = 0; j1 < n1; ++j1)
        for (int b2 = 0; b2 < k2n; ++b2) {
            int k2 = b2 - K[1];
            for (int a = 0; a < k3n; ++a) {
                cplx s = 0;
                for (int j2 = 0; j2 < n2; ++j2)
                    s += t1[((int64_t)j1 * n2 + j2) * k3n + a] * phase((int64_t)k2 * j2, n2);
                t2[((int64_t)j1 * k2n + b2) * k3n + a] = s;
            }
        }
    /* sum over j1 and normalise */
    double inv = 1.0 / ((double)n1 * n2 * n3);
    for (int b1 = 0; b1 < k1n; ++b1) {
        int k1 = b1 - K[0];
        for (int b2 = 0; b2 < k2n; ++b2)
            for (int a = 0; a < k3n; ++a) {
                cplx s = 0;
                for (int j1 = 0; j1 < n1; ++j1)
                    s += t2[((int64_t)j1 * k2n + b2) * k3n + a] * phase((int64_t)k1 * j1, n1);
                out[((int64_t)b1 * k2n + b2) * k3n + a] = s * inv;
            }
    }
    free(t1);
    free(t2);
}

/* ------------------------------------------------------------------ */
/* Hamiltonian data at fixed potential (Section 2.3, (e5) with S = I).  */
/* ------------------------------------------------------------------ */
typedef struct {
    double cell[9], bvec[9], ecut, omega;
    int32_t grid[3], nmax[3], M[3];
    int64_t ng;
    int32_t *miller;  /* ng x 3 */
    double *kin;      /* (1/2)|G|^2 */
    int64_t *pidx;    /* flat index of n mod M on the padded grid */
    double *W;        /* band-limited potential on the padded grid */
    cplx *vt;         /* Vt(k), |k_d| <= 2 nmax_d, C order */
    int32_t nproj;
    cplx *beta;       /* nproj x ng, projector-major */
    double *dkb;      /* KB energies */
    double vmin;
} orc_ham;

static int pow2_at_least(int n)
{
    int m = 1;
    while (m < n) m <<= 1;
    return m;
}

/* Kleinman-Bylander projector in the plane-wave basis (the nonlocal part
 * of the pseudopotential, Section 2.2).  Gaussian radial form of width w,
 * centred at R:  s: exp(-w^2|G|^2/2) exp(-iG.R);  p_alpha: (-i w G_alpha)
 * exp(-w^2|G|^2/2) exp(-iG.R); normalised so that sum_G |beta(G)|^2 = 1. */
static void build_projector(const orc_ham *h, const double *bv, const double *center,
                            int l, int m, double w, cplx *out)
{
    double norm2 = 0.0;
    for (int64_t g = 0; g < h->ng; ++g) {
        double G[3];
        gvec_of(bv, h->miller[3 * g], h->miller[3 * g + 1], h->miller[3 * g + 2], G);
        double g2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
        double gr = G[0] * center[0] + G[1] * center[1] + G[2] * center[2];
        cplx val = exp(-0.5 * w * w * g2) * (cos(gr) - sin(gr) * I);
        if (l == 1) val *= -I * w * G[m];
        out[g] = val;
        norm2 += creal(val) * creal(val) + cimag(val) * cimag(val);
    }
    double s = norm2 > 0 ? 1.0 / sqrt(norm2) : 0.0;
    for (int64_t g = 0; g < h->ng; ++g) out[g] *= s;
}

int32_t orc_ham_create(const double *cell, double ecut, const int32_t *grid, const double *vloc,
                       int32_t nproj, const double *pcenter, const int32_t *pl, const int32_t *pm,
                       const double *pwidth, const double *pd, orc_ham **out)
{
    orc_ham *h = (orc_ham *)calloc(1, sizeof(orc_ham));
    memcpy(h->cell, cell, sizeof(h->cell));
    h->omega = recip(cell, h->bvec);
    h->ecut = ecut;
    memcpy(h->grid, grid, sizeof(h->grid));
    h->ng = orc_sphere(cell, ecut, NULL, 0, h->nmax);
    h->miller = (int32_t *)malloc(sizeof(int32_t) * 3 * h->ng);
    orc_sphere(cell, ecut, h->miller, h->ng, h->nmax);
    for (int d = 0; d < 3; ++d) {
        if (grid[d] < 4 * h->nmax[d] + 1) { free(h->miller); free(h); return -2; }
        h->M[d] = pow2_at_least(4 * h->nmax[d] + 1);
    }
    h->kin = (double *)malloc(sizeof(double) * h->ng);
    h->pidx = (int64_t *)malloc(sizeof(int64_t) * h->ng);
    for (int64_t g = 0; g < h->ng; ++g) {
        double G[3];
        const int32_t *n = h->miller + 3 * g;
        gvec_of(h->bvec, n[0], n[1], n[2], G);
        h->kin[g] = 0.5 * (G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
        int64_t i1 = (n[0] % h->M[0] + h->M[0]) % h->M[0];
        int64_t i2 = (n[1] % h->M[1] + h->M[1]) % h->M[1];
        int64_t i3 = (n[2] % h->M[2] + h->M[2]) % h->M[2];
        h->pidx[g] = (i1 * h->M[1] + i2) * h->M[2] + i3;
    }
    /* Vt on |k_d| <= 2 nmax_d, then the band-limited potential W on the
     * padded grid: W(r) = sum_k Vt(k) exp(+2 pi i k.r/M).  With M_d >=
     * 4 nmax_d + 1 the product W psi has no alias on the sphere, so the FFT
     * apply reproduces sum_n Vt(n_m - n_n) c_n exactly. */
    int32_t K[3] = {2 * h->nmax[0], 2 * h->nmax[1], 2 * h->nmax[2]};
    int k1n = 2 * K[0] + 1, k2n = 2 * K[1] + 1, k3n = 2 * K[2] + 1;
    h->vt = (cplx *)malloc(sizeof(cplx) * (size_t)k1n * k2n * k3n);
    orc_vtilde(grid, vloc, K, h->vt);
    int64_t mtot = (int64_t)h->M[0] * h->M[1] * h->M[2];
    cplx *wc = (cplx *)calloc(mtot, sizeof(cplx));
    for (int b1 = 0; b1 < k1n; ++b1)
        for (int b2 = 0; b2 < k2n; ++b2)
            for (int a = 0; a < k3n; ++a) {
                int64_t i1 = ((b1 - K[0]) % h->M[0] + h->M[0]) % h->M[0];
                int64_t i2 = ((b2 - K[1]) % h->M[1] + h->M[1]) % h->M[1];
                int64_t i3 = ((a - K[2]) % h->M[2] + h->M[2]) % h->M[2];
                wc[(i1 * h->M[1] + i2) * h->M[2] + i3] = h->vt[((int64_t)b1 * k2n + b2) * k3n + a];
            }
    orc_fft3d(wc, h->M, +1);
    h->W = (double *)malloc(sizeof(double) * mtot);
    for (int64_t i = 0; i < mtot; ++i) h->W[i] = creal(wc[i]);
    free(wc);
    int64_t nv = (int64_t)grid[0] * grid[1] * grid[2];
    h->vmin = vloc[0];
    for (int64_t i = 1; i < nv; ++i) if (vloc[i] < h->vmin) h->vmin = vloc[i];
    h->nproj = nproj;
    if (nproj > 0) {
        h->beta = (cplx *)malloc(sizeof(cplx) * (size_t)nproj * h->ng);
        h->dkb = (double *)malloc(sizeof(double) * nproj);
        for (int p = 0; p < nproj; ++p) {
            build_projector(h, h->bvec, pcenter + 3 * p, pl[p], pm[p], pwidth[p], h->beta + (int64_t)p * h->ng);
            h->dkb[p] = pd[p];
        }
    }
    *out = h;
    return 0;
}

void orc_ham_destroy(orc_ham *h)
{
    if (!h) return;
    free(h->miller); free(h->kin); free(h->pidx); free(h->W); free(h->vt);
    free(h->beta); free(h->dkb); free(h);
}

int64_t orc_ham_ng(const orc_ham *h) { return h->ng; }
void orc_ham_info(const orc_ham *h, int32_t *nmax, int32_t *M)
{
    for (int d = 0; d < 3; ++d) { nmax[d] = h->nmax[d]; M[d] = h->M[d]; }
}
void orc_ham_miller(const orc_ham *h, int32_t *out) { memcpy(out, h->miller, sizeof(int32_t) * 3 * h->ng); }
void orc_ham_kin(const orc_ham *h, double *out) { memcpy(out, h->kin, sizeof(double) * h->ng); }
void orc_ham_beta(const orc_ham *h, cplx *out)
{
    if (h->nproj) memcpy(out, h->beta, sizeof(cplx) * h->nproj * h->ng);
}
double orc_ham_vmin(const orc_ham *h) { return h->vmin; }

/* ------------------------------------------------------------------ */
/* H psi (the stiffness matrix of (e5) applied to coefficient vectors): */
/* kinetic (1/2)|G|^2, local potential through the padded-grid FFT,     */
/* nonlocal sum_p D_p beta_p (beta_p^H c); minus shift_b if given.      */
/* ------------------------------------------------------------------ */
static void apply_one(const orc_ham *h, const cplx *c, double shift, cplx *out, cplx *work)
{
    int64_t mtot = (int64_t)h->M[0] * h->M[1] * h->M[2];
    memset(work, 0, sizeof(cplx) * mtot);
    for (int64_t g = 0; g < h->ng; ++g) work[h->pidx[g]] = c[g];
    orc_fft3d(work, h->M, +1);              /* psi(r) = sum_G c_G exp(iG.r) */
    for (int64_t i = 0; i < mtot; ++i) work[i] *= h->W[i];
    orc_fft3d(work, h->M, -1);
    double inv = 1.0 / (double)mtot;
    for (int64_t g = 0; g < h->ng; ++g)
        out[g] = work[h->pidx[g]] * inv + (h->kin[g] - shift) * c[g];
    for (int p = 0; p < h->nproj; ++p) {
        const cplx *bp = h->beta + (int64_t)p * h->ng;
        cplx s = 0;
        for (int64_t g = 0; g < h->ng; ++g) s += conj(bp[g]) * c[g];
        s *= h->dkb[p];
        for (int64_t g = 0; g < h->ng; ++g) out[g] += bp[g] * s;
    }
}

void orc_apply_h(const orc_ham *h, int32_t nb, const cplx *psi, const double *shift, cplx *hpsi)
{
    int64_t mtot = (int64_t)h->M[0] * h->M[1] * h->M[2];
#pragma omp parallel
    {
        cplx *work = (cplx *)malloc(sizeof(cplx) * mtot);
#pragma omp for schedule(dynamic, 1)
        for (int b = 0; b < nb; ++b)
            apply_one(h, psi + (int64_t)b * h->ng, shift ? shift[b] : 0.0, hpsi + (int64_t)b * h->ng, work);
        free(work);
    }
}

/* Dense H (column-major ng x ng) element by element, for tiny cells:
 * h_mn = (1/2)|G_m|^2 delta_mn + Vt(n_m - n_n) + sum_p D_p beta_p(m) conj(beta_p(n)). */
void orc_dense_h(const orc_ham *h, cplx *H)
{
    int32_t K[3] = {2 * h->nmax[0], 2 * h->nmax[1], 2 * h->nmax[2]};
    int k2n = 2 * K[1] + 1, k3n = 2 * K[2] + 1;
    int64_t ng = h->ng;
    for (int64_t n = 0; n < ng; ++n)
        for (int64_t m = 0; m < ng; ++m) {
            const int32_t *a = h->miller + 3 * m, *b = h->miller + 3 * n;
            int64_t d1 = a[0] - b[0] + K[0], d2 = a[1] - b[1] + K[1], d3 = a[2] - b[2] + K[2];
            cplx v = h->vt[(d1 * k2n + d2) * k3n + d3];
            if (m == n) v += h->kin[m];
            for (int p = 0; p < h->nproj; ++p)
                v += h->dkb[p] * h->beta[(int64_t)p * ng + m] * conj(h->beta[(int64_t)p * ng + n]);
            H[m + n * ng] = v;
        }
}

/* ------------------------------------------------------------------ */
/* Small dense linear algebra (column-major).                          */
/* ------------------------------------------------------------------ */
#define A_(i, j) A[(int64_t)(i) + (int64_t)(j) * n]

/* Hermitian eigenproblem by cyclic Jacobi rotations.  A is overwritten;
 * w gets ascending eigenvalues, V (n x n) the matching eigenvectors. */
int32_t orc_heev(int32_t n, cplx *A, double *w, cplx *V)
{
    for (int64_t i = 0; i < (int64_t)n * n; ++i) V[i] = 0;
    for (int i = 0; i < n; ++i) { V[i + (int64_t)i * n] = 1; A_(i, i) = creal(A_(i, i)); }
    int sweep;
    for (sweep = 0; sweep < 60; ++sweep) {
        int rotated = 0;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                cplx apq = A_(p, q);
                double r = cabs(apq);
                double app = creal(A_(p, p)), aqq = creal(A_(q, q));
                if (r <= 1e-17 * sqrt(fabs(app * aqq)) || r < 1e-300) {
                    A_(p, q) = 0; A_(q, p) = 0;
                    continue;
                }
                rotated = 1;
                cplx e = apq / r;                    /* a_pq = r e */
                double theta = (aqq - app) / (2.0 * r);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                cplx ce = conj(e);
                /* A <- A J with J = [[c, s], [-s conj(e), c conj(e)]] on (p,q) */
                for (int k = 0; k < n; ++k) {
                    cplx akp = A_(k, p), akq = A_(k, q);
                    A_(k, p) = c * akp - s * ce * akq;
                    A_(k, q) = s * akp + c * ce * akq;
                }
                /* A <- J^H A */
                for (int k = 0; k < n; ++k) {
                    cplx apk = A_(p, k), aqk = A_(q, k);
                    A_(p, k) = c * apk - s * e * aqk;
                    A_(q, k) = s * apk + c * e * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    cplx vkp = V[k + (int64_t)p * n], vkq = V[k + (int64_t)q * n];
                    V[k + (int64_t)p * n] = c * vkp - s * ce * vkq;
                    V[k + (int64_t)q * n] = s * vkp + c * ce * vkq;
                }
                A_(p, p) = app - t * r;
                A_(q, q) = aqq + t * r;
                A_(p, q) = 0; A_(q, p) = 0;
            }
        if (!rotated) break;
    }
    /* ascending order (selection sort, columns of V follow) */
    for (int i = 0; i < n; ++i) w[i] = creal(A_(i, i));
    for (int i = 0; i < n - 1; ++i) {
        int k = i;
        for (int j = i + 1; j < n; ++j) if (w[j] < w[k]) k = j;
        if (k != i) {
            double t = w[i]; w[i] = w[k]; w[k] = t;
            for (int r = 0; r < n; ++r) {
                cplx x = V[r + (int64_t)i * n];
                V[r + (int64_t)i * n] = V[r + (int64_t)k * n];
                V[r + (int64_t)k * n] = x;
            }
        }
    }
    return sweep;
}

/* Cholesky A = L L^H, L stored in the lower triangle (upper set to 0).
 * Returns 0, or -1 when a pivot is <= 1e-14 * max diagonal entry. */
int32_t orc_cholesky(int32_t n, cplx *A)
{
    double dmax = 0;
    for (int i = 0; i < n; ++i) if (creal(A_(i, i)) > dmax) dmax = creal(A_(i, i));
    for (int j = 0; j < n; ++j) {
        double d = creal(A_(j, j));
        for (int k = 0; k < j; ++k) d -= creal(A_(j, k) * conj(A_(j, k)));
        if (!(d > 1e-14 * dmax)) return -1;
        double ljj = sqrt(d);
        A_(j, j) = ljj;
        for (int i = j + 1; i < n; ++i) {
            cplx s = A_(i, j);
            for (int k = 0; k < j; ++k) s -= A_(i, k) * conj(A_(j, k));
            A_(i, j) = s / ljj;
        }
        for (int i = 0; i < j; ++i) A_(i, j) = 0;
    }
    return 0;
}
#undef A_

/* Solve L X = B in place (L lower, n x n; B n x nrhs). */
static void trsm_lower(int n, const cplx *L, cplx *B, int nrhs)
{
    for (int c = 0; c < nrhs; ++c) {
        cplx *x = B + (int64_t)c * n;
        for (int i = 0; i < n; ++i) {
            cplx s = x[i];
            for (int k = 0; k < i; ++k) s -= L[i + (int64_t)k * n] * x[k];
            x[i] = s / L[i + (int64_t)i * n];
        }
    }
}

/* Solve L^H X = B in place. */
static void trsm_lower_h(int n, const cplx *L, cplx *B, int nrhs)
{
    for (int c = 0; c < nrhs; ++c) {
        cplx *x = B + (int64_t)c * n;
        for (int i = n - 1; i >= 0; --i) {
            cplx s = x[i];
            for (int k = i + 1; k < n; ++k) s -= conj(L[k + (int64_t)i * n]) * x[k];
            x[i] = s / L[i + (int64_t)i * n];
        }
    }
}

/* C = A^H B for band-major blocks A (ma bands), B (mb bands) of length ng;
 * C is ma x mb column-major.  Plain ordered sums. */
static void gram(int64_t ng, int ma, const cplx *A, int mb, const cplx *B, cplx *C)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int j = 0; j < mb; ++j)
        for (int i = 0; i < ma; ++i) {
            const cplx *a = A + (int64_t)i * ng, *b = B + (int64_t)j * ng;
            cplx s = 0;
            for (int64_t g = 0; g < ng; ++g) s += conj(a[g]) * b[g];
            C[i + (int64_t)j * ma] = s;
        }
}

/* Y = X C for band-major X (m bands) and C (m x k column-major). */
static void rotate(int64_t ng, int m, const cplx *X, const cplx *C, int k, cplx *Y)
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < k; ++j) {
        cplx *y = Y + (int64_t)j * ng;
        for (int64_t g = 0; g < ng; ++g) y[g] = 0;
        for (int i = 0; i < m; ++i) {
            cplx cij = C[i + (int64_t)j * m];
            const cplx *x = X + (int64_t)i * ng;
            for (int64_t g = 0; g < ng; ++g) y[g] += x[g] * cij;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Rayleigh-Ritz on span(U) (Algorithm 1, step 4): find the Ritz pairs   */
/* of H in span{u_1..u_m} with orthonormal Ritz vectors.  W = H U.       */
/* S = U^H U, Hs = U^H W, S = L L^H, eig of L^-1 Hs L^-H, C = L^-H Y.    */
/* If S is numerically singular, canonical orthogonalisation:            */
/* S = Q s Q^H, keep s_i > 1e-12 max s, X = Q s^-1/2, eig of X^H Hs X.   */
/* Outputs the lowest nkeep pairs.  Returns flags (ORC_F_CHOL), or -1    */
/* when fewer than nkeep directions survive.                             */
/* ------------------------------------------------------------------ */
int32_t orc_rayleigh_ritz(int64_t ng, int32_t m, int32_t nkeep, const cplx *U, const cplx *W,
                          double *eps, cplx *psi, cplx *hpsi)
{
    cplx *S = (cplx *)malloc(sizeof(cplx) * m * m);
    cplx *Hs = (cplx *)malloc(sizeof(cplx) * m * m);
    cplx *Y = (cplx *)malloc(sizeof(cplx) * m * m);
    cplx *C = (cplx *)calloc((size_t)m * m, sizeof(cplx));
    double *lam = (double *)malloc(sizeof(double) * m);
    int32_t flags = 0;
    gram(ng, m, U, m, U, S);
    gram(ng, m, U, m, W, Hs);
    for (int j = 0; j < m; ++j)
        for (int i = 0; i <= j; ++i) {
            cplx s = 0.5 * (S[i + j * m] + conj(S[j + i * m]));
            cplx h = 0.5 * (Hs[i + j * m] + conj(Hs[j + i * m]));
            S[i + j * m] = s; S[j + i * m] = conj(s);
            Hs[i + j * m] = h; Hs[j + i * m] = conj(h);
        }
    cplx *L = (cplx *)malloc(sizeof(cplx) * m * m);
    memcpy(L, S, sizeof(cplx) * m * m);
    int ncol = m;
    if (orc_cholesky(m, L) == 0) {
        /* Hhat = L^-1 Hs L^-H: X = L^-1 Hs, then Hhat = L^-1 X^H */
        cplx *X = (cplx *)malloc(sizeof(cplx) * m * m);
        memcpy(X, Hs, sizeof(cplx) * m * m);
        trsm_lower(m, L, X, m);
        cplx *Hh = (cplx *)malloc(sizeof(cplx) * m * m);
        for (int j = 0; j < m; ++j)
            for (int i = 0; i < m; ++i) Hh[i + j * m] = conj(X[j + i * m]);
        trsm_lower(m, L, Hh, m);
        for (int j = 0; j < m; ++j)
            for (int i = 0; i <= j; ++i) {
                cplx h = 0.5 * (Hh[i + j * m] + conj(Hh[j + i * m]));
                Hh[i + j * m] = h; Hh[j + i * m] = conj(h);
            }
        orc_heev(m, Hh, lam, Y);
        memcpy(C, Y, sizeof(cplx) * m * m);
        trsm_lower_h(m, L, C, m);       /* C = L^-H Y */
        free(X); free(Hh);
    } else {
        flags |= ORC_F_CHOL;
        cplx *Q = (cplx *)malloc(sizeof(cplx) * m * m);
        double *s = (double *)malloc(sizeof(double) * m);
        cplx *Sc = (cplx *)malloc(sizeof(cplx) * m * m);
        memcpy(Sc, S, sizeof(cplx) * m * m);
        orc_heev(m, Sc, s, Q);
        double smax = s[m - 1];
        int k0 = 0;
        while (k0 < m && !(s[k0] > 1e-12 * smax)) ++k0;
        ncol = m - k0;
        cplx *X = (cplx *)malloc(sizeof(cplx) * m * ncol);
        for (int j = 0; j < ncol; ++j)
            for (int i = 0; i < m; ++i) X[i + j * m] = Q[i + (j + k0) * m] / sqrt(s[j + k0]);
        cplx *T = (cplx *)malloc(sizeof(cplx) * m * ncol);  /* Hs X */
        for (int j = 0; j < ncol; ++j)
            for (int i = 0; i < m; ++i) {
                cplx acc = 0;
                for (int k = 0; k < m; ++k) acc += Hs[i + k * m] * X[k + j * m];
                T[i + j * m] = acc;
            }
        cplx *Hh = (cplx *)malloc(sizeof(cplx) * ncol * ncol);
        for (int j = 0; j < ncol; ++j)
            for (int i = 0; i < ncol; ++i) {
                cplx acc = 0;
                for (int k = 0; k < m; ++k) acc += conj(X[k + i * m]) * T[k + j * m];
                Hh[i + j * ncol] = acc;
            }
        for (int j = 0; j < ncol; ++j)
            for (int i = 0; i <= j; ++i) {
                cplx h = 0.5 * (Hh[i + j * ncol] + conj(Hh[j + i * ncol]));
                Hh[i + j * ncol] = h; Hh[j + i * ncol] = conj(h);
            }
        cplx *Yc = (cplx *)malloc(sizeof(cplx) * ncol * ncol);
        orc_heev(ncol, Hh, lam, Yc);
        for (int j = 0; j < ncol; ++j)
            for (int i = 0; i < m; ++i) {
                cplx acc = 0;
                for (int k = 0; k < ncol; ++k) acc += X[i + k * m] * Yc[k + j * ncol];
                C[i + j * m] = acc;
            }
        free(Q); free(s); free(Sc); free(X); free(T); free(Hh); free(Yc);
    }
    if (ncol < nkeep) {
        free(S); free(Hs); free(Y); free(C); free(lam); free(L);
        return -1;
    }
    for (int i = 0; i < nkeep; ++i) eps[i] = lam[i];
    rotate(ng, m, U, C, nkeep, psi);
    rotate(ng, m, W, C, nkeep, hpsi);
    free(S); free(Hs); free(Y); free(C); free(lam); free(L);
    return flags;
}

/* ------------------------------------------------------------------ */
/* Teter-Payne-Allan preconditioner, x = (1/2)|G|^2 / tau.              */
/* ------------------------------------------------------------------ */
double orc_teter(double x)
{
    double num = 27.0 + 18.0 * x + 12.0 * x * x + 8.0 * x * x * x;
    return num / (num + 16.0 * x * x * x * x);
}

/* ------------------------------------------------------------------ */
/* Source problems of Algorithm 1, step 3, one per band, independent:   */
/*   (H - sigma_b) u_b = (eps_b - sigma_b) psi_b,                       */
/* by preconditioned CG from u = psi, n_cg steps, recurrence residual.  */
/* r0 = eps psi - H psi uses the carried H psi.                          */
/* A band stops on p^H (H - sigma) p <= 0 (flag NEGCURV) or when         */
/* r^H z <= 1e-26 r0^H z0.                                               */
/* mode 1: the correction equation of Algorithm 2, step 3,               */
/*   (H - sigma_b) e_b = -(H psi_b - eps_b psi_b), from e = 0: the same   */
/*   Krylov iteration (r0 is identical), the iterate is e = u - psi       */
/*   accumulated directly instead of formed by a difference.             */
/* mode 2: the projected correction equation of Algorithm 3, step 3,     */
/*   (I - P)(H - sigma_b)(I - P) e_b = (eps_b - H) psi_b, P = psi psi^H /  */
/*   |psi|^2 (the projector onto psi), the shift sigma_b in place of the  */
/*   printed lambda so that the operator is positive definite on the     */
/*   complement of psi: CG from e = 0 in that complement, with the       */
/*   residual, the preconditioned residual and (H - sigma) p projected.   */
/* ------------------------------------------------------------------ */
/* x <- x - psi (psi^H x) / (psi^H psi) */
static void project_out(int64_t ng, const cplx *psi, cplx *x)
{
    cplx c = 0;
    double n = 0;
    for (int64_t g = 0; g < ng; ++g) {
        c += conj(psi[g]) * x[g];
        n += creal(psi[g]) * creal(psi[g]) + cimag(psi[g]) * cimag(psi[g]);
    }
    if (n > 0) {
        c /= n;
        for (int64_t g = 0; g < ng; ++g) x[g] -= c * psi[g];
    }
}

static int32_t pcg_band(const orc_ham *h, const cplx *psi, const cplx *hpsi, double eps, double sigma,
                        int ncg, int mode, cplx *u, cplx *r, cplx *z, cplx *p, cplx *q, cplx *work,
                        double *gamma_hist)
{
    int64_t ng = h->ng;
    double tkin = 0, nrm = 0;
    for (int64_t g = 0; g < ng; ++g) {
        double a2 = creal(psi[g]) * creal(psi[g]) + cimag(psi[g]) * cimag(psi[g]);
        tkin += h->kin[g] * a2;
        nrm += a2;
    }
    double tau = tkin / nrm;
    for (int64_t g = 0; g < ng; ++g) {
        u[g] = mode ? 0 : psi[g];
        r[g] = eps * psi[g] - hpsi[g];
    }
    if (mode == 2) project_out(ng, psi, r);
    for (int64_t g = 0; g < ng; ++g) z[g] = orc_teter(h->kin[g] / tau) * r[g];
    if (mode == 2) project_out(ng, psi, z);
    double gamma = 0;
    for (int64_t g = 0; g < ng; ++g) {
        p[g] = z[g];
        gamma += creal(conj(r[g]) * z[g]);
    }
    if (gamma_hist) gamma_hist[0] = gamma;
    double gamma0 = gamma;
    int32_t flags = 0;
    if (!(gamma0 > 0)) return isnan(gamma0) ? ORC_F_NAN : 0;
    for (int k = 1; k <= ncg; ++k) {
        apply_one(h, p, sigma, q, work);
        if (mode == 2) project_out(ng, psi, q);
        double pq = 0;
        for (int64_t g = 0; g < ng; ++g) pq += creal(conj(p[g]) * q[g]);
        if (!(pq > 0)) { flags |= isnan(pq) ? ORC_F_NAN : ORC_F_NEGCURV; break; }
        double alpha = gamma / pq;
        for (int64_t g = 0; g < ng; ++g) {
            u[g] += alpha * p[g];
            r[g] -= alpha * q[g];
            z[g] = orc_teter(h->kin[g] / tau) * r[g];
        }
        if (mode == 2) project_out(ng, psi, z);
        double gnew = 0;
        for (int64_t g = 0; g < ng; ++g) gnew += creal(conj(r[g]) * z[g]);
        if (gamma_hist) gamma_hist[k] = gnew;
        if (gnew <= 1e-26 * gamma0) break;
        double beta = gnew / gamma;
        for (int64_t g = 0; g < ng; ++g) p[g] = z[g] + beta * p[g];
        gamma = gnew;
    }
    return flags;
}

int32_t orc_pcg(const orc_ham *h, int32_t nb, const cplx *psi, const cplx *hpsi, const double *eps,
                const double *shift, int32_t ncg, int32_t mode, cplx *u, int32_t *flags,
                double *gamma_hist)
{
    int64_t ng = h->ng, mtot = (int64_t)h->M[0] * h->M[1] * h->M[2];
    int32_t all = 0;
#pragma omp parallel reduction(| : all)
    {
        cplx *r = (cplx *)malloc(sizeof(cplx) * ng), *z = (cplx *)malloc(sizeof(cplx) * ng);
        cplx *p = (cplx *)malloc(sizeof(cplx) * ng), *q = (cplx *)malloc(sizeof(cplx) * ng);
        cplx *work = (cplx *)malloc(sizeof(cplx) * mtot);
#pragma omp for schedule(dynamic, 1)
        for (int b = 0; b < nb; ++b) {
            int32_t f = pcg_band(h, psi + (int64_t)b * ng, hpsi + (int64_t)b * ng, eps[b], shift[b], ncg,
                                 mode, u + (int64_t)b * ng, r, z, p, q, work,
                                 gamma_hist ? gamma_hist + (int64_t)b * (ncg + 1) : NULL);
            if (flags) flags[b] = f;
            all |= f;
        }
        free(r); free(z); free(p); free(q); free(work);
    }
    return all;
}

/* ------------------------------------------------------------------ */
/* Lower bound of the spectrum (Weyl): kinetic >= 0, the local part is  */
/* a compression of multiplication by V so >= min_j V_j, and the        */
/* nonlocal part B D B^H has the nonzero eigenvalues of L^H D L with    */
/* B^H B = L L^H.  sigma_lb = min V + min(0, lambda_min(V_NL)) - 0.1.   */
/* ------------------------------------------------------------------ */
double orc_nl_min_eig(const orc_ham *h)
{
    int np = h->nproj;
    if (np == 0) return 0.0;
    cplx *G = (cplx *)malloc(sizeof(cplx) * np * np);
    gram(h->ng, np, h->beta, np, h->beta, G);
    if (orc_cholesky(np, G) != 0) { free(G); return NAN; }
    cplx *Mx = (cplx *)malloc(sizeof(cplx) * np * np);
    for (int j = 0; j < np; ++j)
        for (int i = 0; i < np; ++i) {
            cplx acc = 0; /* (L^H D L)_ij = sum_k conj(L_ki) D_k L_kj */
            for (int k = 0; k < np; ++k) acc += conj(G[k + i * np]) * h->dkb[k] * G[k + j * np];
            Mx[i + j * np] = acc;
        }
    double *w = (double *)malloc(sizeof(double) * np);
    cplx *V = (cplx *)malloc(sizeof(cplx) * np * np);
    orc_heev(np, Mx, w, V);
    double lmin = w[0];
    free(G); free(Mx); free(w); free(V);
    return lmin;
}

double orc_shift_bound(const orc_ham *h)
{
    double lnl = orc_nl_min_eig(h);
    return h->vmin + (lnl < 0 ? lnl : 0.0) - 0.1;
}

/* ------------------------------------------------------------------ */
/* Residual norms |H psi_b - eps_b psi_b|.                               */
/* ------------------------------------------------------------------ */
static void residual_norms(int64_t ng, int nb, const cplx *psi, const cplx *hpsi, const double *eps,
                           double *res)
{
    for (int b = 0; b < nb; ++b) {
        double s = 0;
        for (int64_t g = 0; g < ng; ++g) {
            cplx d = hpsi[(int64_t)b * ng + g] - eps[b] * psi[(int64_t)b * ng + g];
            s += creal(d) * creal(d) + cimag(d) * cimag(d);
        }
        res[b] = sqrt(s);
    }
}

void orc_residual_norms(int64_t ng, int32_t nb, const cplx *psi, const cplx *hpsi, const double *eps,
                        double *res)
{
    residual_norms(ng, nb, psi, hpsi, eps, res);
}

/* ------------------------------------------------------------------ */
/* ParO at fixed cutoff and potential (Algorithm 1 with steps 1, 3, 4,  */
/* 5; the cutoff is not raised).  variant 0: Algorithm 1, RR on the      */
/* source solutions u; variant 1: Algorithm 2 (MParO I), RR on           */
/* span{psi, e} with e the solution of the correction equation         */
/* (H - sigma) e = -(H psi - eps psi) (e = u - psi), normalised;          */
/* variant 2: Algorithm 3 (MParO II), the same with e from the           */
/* projected correction equation (pcg_band mode 2).                       */
/*                                                                       */
/* psi: in the trial block, out the Ritz vectors (nb bands).             */
/* shift_mode 0: sigma = sigma_lb for every step.                        */
/* shift_mode 1: sigma = max(sigma_lb, eps_1 - 0.05 - |r_1|) when        */
/*   |r_1| < 0.1, else sigma_lb; on a NEGCURV flag the outer iteration    */
/*   is redone with sigma_lb.                                             */
/* Histories: eps_hist and res_hist (n_outer+1) x nb, sigma_hist n_outer. */
/* Returns the OR of all flags.                                           */
/* ------------------------------------------------------------------ */
int32_t orc_paro(const orc_ham *h, int32_t nb, cplx *psi, cplx *hpsi, double *eps,
                 int32_t n_outer, int32_t ncg, int32_t variant, int32_t shift_mode, double sigma_lb,
                 double *eps_hist, double *res_hist, double *sigma_hist)
{
    int64_t ng = h->ng;
    int32_t all = 0;
    int m = variant >= 1 ? 2 * nb : nb;
    cplx *U = (cplx *)malloc(sizeof(cplx) * ng * m);
    cplx *W = (cplx *)malloc(sizeof(cplx) * ng * m);
    double *sig = (double *)malloc(sizeof(double) * nb);
    int32_t *fl = (int32_t *)malloc(sizeof(int32_t) * nb);
    double *res = (double *)malloc(sizeof(double) * nb);
    /* step 1: initial (eps^0, psi^0) by Rayleigh-Ritz on the trial block */
    memcpy(U, psi, sizeof(cplx) * ng * nb);
    orc_apply_h(h, nb, U, NULL, W);
    int32_t f = orc_rayleigh_ritz(ng, nb, nb, U, W, eps, psi, hpsi);
    if (f < 0) goto done;
    all |= f;
    residual_norms(ng, nb, psi, hpsi, eps, res);
    if (eps_hist) memcpy(eps_hist, eps, sizeof(double) * nb);
    if (res_hist) memcpy(res_hist, res, sizeof(double) * nb);
    for (int it = 0; it < n_outer; ++it) {
        double sigma = sigma_lb;
        if (shift_mode == 1 && res[0] < 0.1) {
            double s = eps[0] - 0.05 - res[0];
            if (s > sigma) sigma = s;
        }
        /* Algorithm 1: u into U[0:nb]; Algorithms 2 and 3: e into U[nb:2nb] */
        cplx *sol = variant >= 1 ? U + ng * nb : U;
        for (int attempt = 0; attempt < 2; ++attempt) {
            for (int b = 0; b < nb; ++b) sig[b] = sigma;
            int32_t pf = orc_pcg(h, nb, psi, hpsi, eps, sig, ncg, variant, sol, fl, NULL);
            if ((pf & ORC_F_NEGCURV) && sigma != sigma_lb) { sigma = sigma_lb; all |= ORC_F_NEGCURV; continue; }
            all |= pf;
            break;
        }
        if (sigma_hist) sigma_hist[it] = sigma;
        if (variant >= 1) {
            /* U = [psi, e/|e|]; W = [H psi, H e] */
            cplx *E = U + ng * nb;
            for (int b = 0; b < nb; ++b) {
                double s = 0;
                for (int64_t g = 0; g < ng; ++g) {
                    cplx d = E[(int64_t)b * ng + g];
                    s += creal(d) * creal(d) + cimag(d) * cimag(d);
                }
                s = s > 0 ? 1.0 / sqrt(s) : 0.0;
                for (int64_t g = 0; g < ng; ++g) E[(int64_t)b * ng + g] *= s;
            }
            memcpy(U, psi, sizeof(cplx) * ng * nb);
            memcpy(W, hpsi, sizeof(cplx) * ng * nb);
            orc_apply_h(h, nb, E, NULL, W + ng * nb);
        } else {
            orc_apply_h(h, nb, U, NULL, W);
        }
        f = orc_rayleigh_ritz(ng, m, nb, U, W, eps, psi, hpsi);
        if (f < 0) { all |= ORC_F_CHOL; break; }
        all |= f;
        residual_norms(ng, nb, psi, hpsi, eps, res);
        if (eps_hist) memcpy(eps_hist + (int64_t)(it + 1) * nb, eps, sizeof(double) * nb);
        if (res_hist) memcpy(res_hist + (int64_t)(it + 1) * nb, res, sizeof(double) * nb);
    }
done:
    free(U); free(W); free(sig); free(fl); free(res);
    return all;
}

/* ------------------------------------------------------------------ */
/* Electron density on the FFT grid (the quantity the Hellmann-Feynman    */
/* derivative of the eigenvalue sum needs):                               */
/*   rho_j = sum_b w_b |psi_b(r_j)|^2,                                    */
/*   psi_b(r_j) = sum_G c_bG exp(2 pi i n.j / N)  (eq. (e2) at the grid   */
/*   point r_j = sum_d (j_d / N_d) a_d, without the 1 / sqrt(Omega)).     */
/* d(sum_b w_b eps_b) / dV_j = rho_j / (N1 N2 N3) for eigenpairs, since   */
/* the matrix element of eq. (e5) is the grid sum                         */
/* (1/N) sum_j V_j exp(-2 pi i (n_m - n_n).j / N).                        */
/* Direct separable sums over n3, n2, n1 (no FFT).  Output C order        */
/* [j1][j2][j3]; bands summed in order.                                   */
/* ------------------------------------------------------------------ */
void orc_density(const orc_ham *h, int32_t nb, const cplx *psi, const double *w, double *rho)
{
    const int N1 = h->grid[0], N2 = h->grid[1], N3 = h->grid[2];
    const int m1 = h->nmax[0], m2 = h->nmax[1];
    const int L1 = 2 * m1 + 1, L2 = 2 * m2 + 1;
    const int64_t nv = (int64_t)N1 * N2 * N3;
    cplx *t1 = (cplx *)malloc(sizeof(cplx) * N1), *t2 = (cplx *)malloc(sizeof(cplx) * N2);
    cplx *t3 = (cplx *)malloc(sizeof(cplx) * N3);
    for (int k = 0; k < N1; ++k) t1[k] = cexp(I * TWO_PI * k / N1);
    for (int k = 0; k < N2; ++k) t2[k] = cexp(I * TWO_PI * k / N2);
    for (int k = 0; k < N3; ++k) t3[k] = cexp(I * TWO_PI * k / N3);
    double *per = (double *)calloc((size_t)nb * nv, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < nb; ++b) {
        const cplx *c = psi + (int64_t)b * h->ng;
        /* A[n1][n2][j3] = sum_n3 c exp(2 pi i n3 j3 / N3) */
        cplx *A = (cplx *)calloc((size_t)L1 * L2 * N3, sizeof(cplx));
        for (int64_t g = 0; g < h->ng; ++g) {
            const int n1 = h->miller[3 * g], n2 = h->miller[3 * g + 1], n3 = h->miller[3 * g + 2];
            cplx *a = A + ((int64_t)(n1 + m1) * L2 + (n2 + m2)) * N3;
            for (int j3 = 0; j3 < N3; ++j3) a[j3] += c[g] * t3[(((int64_t)n3 * j3) % N3 + N3) % N3];
        }
        /* B[n1][j2][j3] = sum_n2 A exp(2 pi i n2 j2 / N2) */
        cplx *B = (cplx *)calloc((size_t)L1 * N2 * N3, sizeof(cplx));
        for (int i1 = 0; i1 < L1; ++i1)
            for (int i2 = 0; i2 < L2; ++i2) {
                const cplx *a = A + ((int64_t)i1 * L2 + i2) * N3;
                const int n2 = i2 - m2;
                for (int j2 = 0; j2 < N2; ++j2) {
                    const cplx e = t2[(((int64_t)n2 * j2) % N2 + N2) % N2];
                    cplx *bb = B + ((int64_t)i1 * N2 + j2) * N3;
                    for (int j3 = 0; j3 < N3; ++j3) bb[j3] += a[j3] * e;
                }
            }
        /* psi[j1][j2][j3] = sum_n1 B exp(2 pi i n1 j1 / N1); |psi|^2 */
        double *out = per + (int64_t)b * nv;
        for (int j1 = 0; j1 < N1; ++j1)
            for (int j2 = 0; j2 < N2; ++j2)
                for (int j3 = 0; j3 < N3; ++j3) {
                    cplx acc = 0;
                    for (int i1 = 0; i1 < L1; ++i1) {
                        const int n1 = i1 - m1;
                        acc += B[((int64_t)i1 * N2 + j2) * N3 + j3] * t1[(((int64_t)n1 * j1) % N1 + N1) % N1];
                    }
                    out[((int64_t)j1 * N2 + j2) * N3 + j3] = creal(acc) * creal(acc) + cimag(acc) * cimag(acc);
                }
        free(A);
        free(B);
    }
    for (int64_t j = 0; j < nv; ++j) {
        double s = 0;
        for (int b = 0; b < nb; ++b) s += (w ? w[b] : 1.0) * per[(int64_t)b * nv + j];
        rho[j] = s;
    }
    free(per); free(t1); free(t2); free(t3);
}

/* ------------------------------------------------------------------ */
/* Hellmann-Feynman derivatives of sum_b w_b <psi_b| V_NL |psi_b> with   */
/* respect to the KB energies d_p and the projector centres R_p, where  */
/* V_NL = sum_p d_p beta_p beta_p^H (Section 2.2) and beta_p(G) carries  */
/* the phase exp(-i G.R_p):                                              */
/*   dd[p]       = sum_b w_b |P_pb|^2,       P_pb = beta_p^H psi_b,     */
/*   dR[3p + a]  = sum_b w_b d_p 2 Re(conj(P_pb) Q_pb^a),               */
/*   Q_pb^a      = (d beta_p / d R_a)^H psi_b,  d beta_p / d R_a = -i G_a beta_p. */
/* For eigenpairs these are the derivatives of sum_b w_b eps_b.         */
/* ------------------------------------------------------------------ */
void orc_projector_gradient(const orc_ham *h, int32_t nb, const cplx *psi, const double *w, double *dd,
                            double *dR)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int p = 0; p < h->nproj; ++p) {
        const cplx *bp = h->beta + (int64_t)p * h->ng;
        double sd = 0.0, sr[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < nb; ++b) {
            const cplx *c = psi + (int64_t)b * h->ng;
            cplx P = 0, Q[3] = {0, 0, 0};
            for (int64_t g = 0; g < h->ng; ++g) {
                double G[3];
                gvec_of(h->bvec, h->miller[3 * g], h->miller[3 * g + 1], h->miller[3 * g + 2], G);
                P += conj(bp[g]) * c[g];
                for (int a = 0; a < 3; ++a) Q[a] += conj(-I * G[a] * bp[g]) * c[g];
            }
            const double wb = w ? w[b] : 1.0;
            sd += wb * (creal(P) * creal(P) + cimag(P) * cimag(P));
            for (int a = 0; a < 3; ++a) sr[a] += wb * h->dkb[p] * 2.0 * creal(conj(P) * Q[a]);
        }
        dd[p] = sd;
        for (int a = 0; a < 3; ++a) dR[3 * p + a] = sr[a];
    }
}

int32_t orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
