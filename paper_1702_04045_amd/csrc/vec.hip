// Band-wise vector kernels: the preconditioned CG of the source problems
// (Algorithm 1, step 3), residual norms (step 5) and the correction vectors
// of Algorithm 2.  Every reduction goes through per-work-group partial sums
// that the consumer adds in a fixed order, so runs are bitwise reproducible.
#include <algorithm>
#include <cstring>

#include "fft_device.h"
#include "group.h"
#include "paro_internal.h"
#include "reduce_device.h"

namespace paro {

namespace {

constexpr int kVecThreads = 256;
constexpr int kVecChunk = 2048;  // sphere points per work-group

__device__ __forceinline__ double sum_parts(const double *p, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += p[i];
    return s;
}

// Teter-Payne-Allan preconditioner K(x), x = (1/2)|G|^2 / tau.
__device__ __forceinline__ double teter(double x)
{
    const double num = 27.0 + 18.0 * x + 12.0 * x * x + 8.0 * x * x * x;
    return num / (num + 16.0 * x * x * x * x);
}

// partial sums of <psi|T|psi> and <psi|psi>
__device__ __forceinline__ void pcg_init_parts_body(int bx, int by, int64_t ng, const double2 *__restrict__ psi,
                                                    int64_t ld, const double *__restrict__ kin,
                                                    double *__restrict__ dots, int nb)
{
    __shared__ double red[kVecThreads / 64];
    const int band = by;
    const double2 *x = psi + band * ld;
    double tk = 0.0, nr = 0.0;
    const int64_t g0 = (int64_t)bx * kVecChunk;
    const int64_t g1 = g0 + kVecChunk < ng ? g0 + kVecChunk : ng;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kVecThreads) {
        const double2 v = x[g];
        const double a2 = v.x * v.x + v.y * v.y;
        tk += kin[g] * a2;
        nr += a2;
    }
    tk = block_sum<kVecThreads>(tk, red);
    nr = block_sum<kVecThreads>(nr, red);
    if (threadIdx.x == 0) {
        dots[((size_t)DOT_TKIN * nb + band) * kMaxParts + bx] = tk;
        dots[((size_t)DOT_NRM * nb + band) * kMaxParts + bx] = nr;
    }
}
__global__ void __launch_bounds__(kVecThreads)
k_pcg_init_parts(int64_t ng, const double2 *__restrict__ psi, int64_t ld, const double *__restrict__ kin,
                 double *__restrict__ dots, int nb)
{
    pcg_init_parts_body(blockIdx.x, blockIdx.y, ng, psi, ld, kin, dots, nb);
}
__global__ void __launch_bounds__(kVecThreads) k_pcg_init_parts_grp(GroupTab t)
{
    int e, bx, by;
    group_block(t, e, bx, by);
    const PcgInitPartsArgs &a = *static_cast<const PcgInitPartsArgs *>(t.args[e]);
    pcg_init_parts_body(bx, by, a.ng, a.psi, a.ld, a.kin, a.dots, a.nb);
}

// u = psi (correction: u = 0, the iterate is then e = u - psi of the
// correction equation of Algorithm 2); r = eps psi - H psi; z = K r;
// partial r^H z.  r is formed in FP64 from the FP64 psi and H psi; the
// vectors are stored as CV (double2, or float2 in the mixed-precision
// solve) and u as CU.
template <class CV, class CU>
__device__ __forceinline__ void pcg_init_body(int bx, int by, int64_t ng, int nparts, const double2 *__restrict__ psi,
                                              const double2 *__restrict__ hpsi, int64_t ld,
                                              const double *__restrict__ eps, const double *__restrict__ kin,
                                              CU *__restrict__ u, int64_t ldu, CV *__restrict__ r,
                                              CV *__restrict__ z, int64_t ldv, double *__restrict__ dots,
                                              double *__restrict__ sc, int nb, int correction)
{
    __shared__ double red[kVecThreads / 64];
    const int band = by;
    const double tk = sum_parts(dots + ((size_t)DOT_TKIN * nb + band) * kMaxParts, nparts);
    const double nr = sum_parts(dots + ((size_t)DOT_NRM * nb + band) * kMaxParts, nparts);
    const double tau = tk / nr;
    if (bx == 0 && threadIdx.x == 0) sc[SC_TAU * nb + band] = tau;
    const double e = eps[band];
    const double2 *x = psi + band * ld, *hx = hpsi + band * ld;
    CU *uu = u + band * ldu;
    CV *rr = r + band * ldv, *zz = z + band * ldv;
    double rz = 0.0;
    const int64_t g0 = (int64_t)bx * kVecChunk;
    const int64_t g1 = g0 + kVecChunk < ng ? g0 + kVecChunk : ng;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kVecThreads) {
        const double2 v = x[g], hv = hx[g];
        const CV rv = cmk<CV>(e * v.x - hv.x, e * v.y - hv.y);
        const double k = teter(kin[g] / tau);
        const CV zv = cmk<CV>(k * rv.x, k * rv.y);
        uu[g] = correction ? cmk<CU>(0.0, 0.0) : cmk<CU>(v.x, v.y);
        rr[g] = rv;
        zz[g] = zv;
        rz += (double)rv.x * (double)zv.x + (double)rv.y * (double)zv.y;
    }
    rz = block_sum<kVecThreads>(rz, red);
    if (threadIdx.x == 0) dots[((size_t)DOT_RZ * nb + band) * kMaxParts + bx] = rz;
}
template <class CV, class CU>
__global__ void __launch_bounds__(kVecThreads)
k_pcg_init(int64_t ng, int nparts, const double2 *__restrict__ psi, const double2 *__restrict__ hpsi, int64_t ld,
           const double *__restrict__ eps, const double *__restrict__ kin, CU *__restrict__ u, int64_t ldu,
           CV *__restrict__ r, CV *__restrict__ z, int64_t ldv, double *__restrict__ dots,
           double *__restrict__ sc, int nb, int correction)
{
    pcg_init_body<CV, CU>(blockIdx.x, blockIdx.y, ng, nparts, psi, hpsi, ld, eps, kin, u, ldu, r, z, ldv, dots, sc,
                          nb, correction);
}
template <class CV, class CU> __global__ void __launch_bounds__(kVecThreads) k_pcg_init_grp(GroupTab t)
{
    int e, bx, by;
    group_block(t, e, bx, by);
    const PcgInitArgs<CV, CU> &a = *static_cast<const PcgInitArgs<CV, CU> *>(t.args[e]);
    pcg_init_body<CV, CU>(bx, by, a.ng, a.nparts, a.psi, a.hpsi, a.ld, a.eps, a.kin, a.u, a.ldu, a.r, a.z, a.ldv,
                          a.dots, a.sc, a.nb, a.correction);
}

// alpha = gamma / p^H q; u += alpha p; r -= alpha q; z = K r; partial r^H z
// (FP64 arithmetic on CV / CU storage).
template <class CV, class CU>
__device__ __forceinline__ void pcg_update_body(int bx, int by, int64_t ng, int npq, const CV *__restrict__ p,
                                                const CV *__restrict__ q, int64_t ldv, CU *__restrict__ u,
                                                int64_t ldu, CV *__restrict__ r, CV *__restrict__ z,
                                                const double *__restrict__ kin, const double *__restrict__ dots_pq,
                                                double *__restrict__ dots_rz, const double *__restrict__ sc,
                                                const int32_t *__restrict__ active, int nb)
{
    __shared__ double red[kVecThreads / 64];
    const int band = by;
    const double pq = sum_parts(dots_pq + (size_t)band * kMaxParts, npq) + sc[SC_NLQ * nb + band];
    const bool go = active[band] && pq > 0.0;
    double rz = 0.0;
    if (go) {
        const double alpha = sc[SC_GAMMA * nb + band] / pq;
        const double tau = sc[SC_TAU * nb + band];
        const CV *pp = p + band * ldv, *qq = q + band * ldv;
        CU *uu = u + band * ldu;
        CV *rr = r + band * ldv, *zz = z + band * ldv;
        const int64_t g0 = (int64_t)bx * kVecChunk;
        const int64_t g1 = g0 + kVecChunk < ng ? g0 + kVecChunk : ng;
        for (int64_t g = g0 + threadIdx.x; g < g1; g += kVecThreads) {
            const CV pv = pp[g], qv = qq[g];
            const CU uv = uu[g];
            const CV rv0 = rr[g];
            const double rx = rv0.x - alpha * qv.x, ry = rv0.y - alpha * qv.y;
            const CV rv = cmk<CV>(rx, ry);
            const double k = teter(kin[g] / tau);
            const CV zv = cmk<CV>(k * rv.x, k * rv.y);
            uu[g] = cmk<CU>(uv.x + alpha * pv.x, uv.y + alpha * pv.y);
            rr[g] = rv;
            zz[g] = zv;
            rz += (double)rv.x * (double)zv.x + (double)rv.y * (double)zv.y;
        }
    }
    rz = block_sum<kVecThreads>(rz, red);
    if (threadIdx.x == 0) dots_rz[(size_t)band * kMaxParts + bx] = rz;
}
template <class CV, class CU>
__global__ void __launch_bounds__(kVecThreads)
k_pcg_update(int64_t ng, int npq, const CV *__restrict__ p, const CV *__restrict__ q, int64_t ldv,
             CU *__restrict__ u, int64_t ldu, CV *__restrict__ r, CV *__restrict__ z,
             const double *__restrict__ kin, const double *__restrict__ dots_pq, double *__restrict__ dots_rz,
             const double *__restrict__ sc, const int32_t *__restrict__ active, int nb)
{
    pcg_update_body<CV, CU>(blockIdx.x, blockIdx.y, ng, npq, p, q, ldv, u, ldu, r, z, kin, dots_pq, dots_rz, sc,
                            active, nb);
}
template <class CV, class CU> __global__ void __launch_bounds__(kVecThreads) k_pcg_update_grp(GroupTab t)
{
    int e, bx, by;
    group_block(t, e, bx, by);
    const PcgUpdateArgs<CV, CU> &a = *static_cast<const PcgUpdateArgs<CV, CU> *>(t.args[e]);
    pcg_update_body<CV, CU>(bx, by, a.ng, a.npq, a.p, a.q, a.ldv, a.u, a.ldu, a.r, a.z, a.kin, a.dots_pq,
                            a.dots_rz, a.sc, a.active, a.nb);
}

// u_b = base_b + d_b (base != null) or u_b = d_b, in FP64
__global__ void __launch_bounds__(kVecThreads)
k_finish_correction(int64_t ng, const double2 *__restrict__ base, int64_t ld, const float2 *__restrict__ d,
                    int64_t ldv, double2 *__restrict__ u, int64_t ldu)
{
    const int band = blockIdx.y;
    const int64_t g0 = (int64_t)blockIdx.x * kVecChunk;
    const int64_t g1 = g0 + kVecChunk < ng ? g0 + kVecChunk : ng;
    const float2 *dd = d + band * ldv;
    double2 *uu = u + band * ldu;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kVecThreads) {
        const float2 dv = dd[g];
        double2 o = make_double2(dv.x, dv.y);
        if (base) {
            const double2 b = base[band * ld + g];
            o.x += b.x;
            o.y += b.y;
        }
        uu[g] = o;
    }
}

// Partial sums of psi^H x (re, im) and |psi|^2 (projection onto the
// complement of psi, Algorithm 3).
__global__ void __launch_bounds__(kVecThreads)
k_proj_parts(int64_t ng, const double2 *__restrict__ psi, int64_t ld, const double2 *__restrict__ x, int64_t ldx,
             double *__restrict__ dots, int nb)
{
    __shared__ double red[kVecThreads / 64];
    const int band = blockIdx.y;
    const double2 *pp = psi + band * ld, *xx = x + band * ldx;
    double cr = 0.0, ci = 0.0, nn = 0.0;
    const int64_t g0 = (int64_t)blockIdx.x * kVecChunk;
    const int64_t g1 = g0 + kVecChunk < ng ? g0 + kVecChunk : ng;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kVecThreads) {
        const double2 a = pp[g], b = xx[g];
        cr += a.x * b.x + a.y * b.y;
        ci += a.x * b.y - a.y * b.x;
        nn += a.x * a.x + a.y * a.y;
    }
    cr = block_sum<kVecThreads>(cr, red);
    ci = block_sum<kVecThreads>(ci, red);
    nn = block_sum<kVecThreads>(nn, red);
    if (threadIdx.x == 0) {
        dots[((size_t)DOT_PJR * nb + band) * kMaxParts + blockIdx.x] = cr;
        dots[((size_t)DOT_PJI * nb + band) * kMaxParts + blockIdx.x] = ci;
        dots[((size_t)DOT_PJN * nb + band) * kMaxParts + blockIdx.x] = nn;
    }
}

// x <- x - c psi, c = psi^H x / |psi|^2 from k_proj_parts.  zout != null:
// zout = K x (x is a residual); rref != null: partial Re(rref^H x) into
// dots_rz (x is a preconditioned residual).
__global__ void __launch_bounds__(kVecThreads)
k_proj_sub(int64_t ng, int nparts, const double2 *__restrict__ psi, int64_t ld, double2 *__restrict__ x,
           int64_t ldx, const double *__restrict__ dots, int nb, const double *__restrict__ kin,
           const double *__restrict__ sc, double2 *__restrict__ zout, const double2 *__restrict__ rref,
           double *__restrict__ dots_rz)
{
    __shared__ double red[kVecThreads / 64];
    const int band = blockIdx.y;
    const double cr = sum_parts(dots + ((size_t)DOT_PJR * nb + band) * kMaxParts, nparts);
    const double ci = sum_parts(dots + ((size_t)DOT_PJI * nb + band) * kMaxParts, nparts);
    const double nn = sum_parts(dots + ((size_t)DOT_PJN * nb + band) * kMaxParts, nparts);
    const double s = nn > 0.0 ? 1.0 / nn : 0.0;
    const double c_r = cr * s, c_i = ci * s;
    const double tau = zout ? sc[SC_TAU * nb + band] : 1.0;
    const double2 *pp = psi + band * ld;
    double2 *xx = x + band * ldx;
    double rz = 0.0;
    const int64_t g0 = (int64_t)blockIdx.x * kVecChunk;
    const int64_t g1 = g0 + kVecChunk < ng ? g0 + kVecChunk : ng;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kVecThreads) {
        const double2 a = pp[g];
        double2 v = xx[g];
        v.x -= c_r * a.x - c_i * a.y;
        v.y -= c_r * a.y + c_i * a.x;
        xx[g] = v;
        if (zout) {
            const double k = teter(kin[g] / tau);
            zout[band * ldx + g] = make_double2(k * v.x, k * v.y);
        }
        if (rref) {
            const double2 r = rref[band * ldx + g];
            rz += r.x * v.x + r.y * v.y;
        }
    }
    if (rref) {
        rz = block_sum<kVecThreads>(rz, red);
        if (threadIdx.x == 0) dots_rz[(size_t)band * kMaxParts + blockIdx.x] = rz;
    }
}

// Per-band PCG scalars.
// stage 0 (after init): gamma = gamma0 = r^H z; active = gamma0 > 0.
// stage 1 (after an update): stop on p^H q <= 0 (flag NEGCURV, or NAN), else
//   gamma' = r^H z; stop when gamma' <= 1e-26 gamma0, else beta = gamma'/gamma.
__device__ __forceinline__ void pcg_scalars_body(int nb, int stage, int nparts_rz, int npq,
                                                 const double *__restrict__ dots_pq,
                                                 const double *__restrict__ dots_rz, double *__restrict__ sc,
                                                 int32_t *__restrict__ active, int32_t *__restrict__ bflags,
                                                 int32_t *__restrict__ band_flags_out, int32_t *__restrict__ status)
{
    for (int b = threadIdx.x; b < nb; b += kVecThreads) {
        const double rz = sum_parts(dots_rz + (size_t)b * kMaxParts, nparts_rz);
        if (stage == 0) {
            sc[SC_GAMMA * nb + b] = rz;
            sc[SC_GAMMA0 * nb + b] = rz;
            sc[SC_BETA * nb + b] = 0.0;
            sc[SC_NLQ * nb + b] = 0.0;
            const bool ok = rz > 0.0;
            active[b] = ok ? 1 : 0;
            const int32_t f = (rz != rz) ? PARO_F_NAN : 0;
            bflags[b] = f;
            if (f) atomicOr(status, f);
        } else if (active[b]) {
            const double pq = sum_parts(dots_pq + (size_t)b * kMaxParts, npq) + sc[SC_NLQ * nb + b];
            if (!(pq > 0.0)) {
                const int32_t f = (pq != pq) ? PARO_F_NAN : PARO_F_NEGCURV;
                active[b] = 0;
                bflags[b] |= f;
                atomicOr(status, f);
            } else if (rz != rz) {
                active[b] = 0;
                bflags[b] |= PARO_F_NAN;
                atomicOr(status, PARO_F_NAN);
            } else if (rz <= 1e-26 * sc[SC_GAMMA0 * nb + b]) {
                active[b] = 0;
            } else {
                sc[SC_BETA * nb + b] = rz / sc[SC_GAMMA * nb + b];
                sc[SC_GAMMA * nb + b] = rz;
            }
        }
        if (band_flags_out) band_flags_out[b] = bflags[b];
    }
}
__global__ void __launch_bounds__(kVecThreads)
k_pcg_scalars(int nb, int stage, int nparts_rz, int npq, const double *__restrict__ dots_pq,
              const double *__restrict__ dots_rz, double *__restrict__ sc, int32_t *__restrict__ active,
              int32_t *__restrict__ bflags, int32_t *__restrict__ band_flags_out, int32_t *__restrict__ status)
{
    pcg_scalars_body(nb, stage, nparts_rz, npq, dots_pq, dots_rz, sc, active, bflags, band_flags_out, status);
}
// one work-group per entry
__global__ void __launch_bounds__(kVecThreads) k_pcg_scalars_grp(GroupTab t, int stage)
{
    const PcgScalarsArgs &a = *static_cast<const PcgScalarsArgs *>(t.args[blockIdx.x]);
    pcg_scalars_body(a.nb, stage, a.nparts_rz, a.npq, a.dots_pq, a.dots_rz, a.sc, a.active, a.bflags,
                     a.band_flags_out, a.status);
}

// partial sums of |hpsi - eps psi|^2
__device__ __forceinline__ void res_parts_body(int bx, int by, int64_t ng, const double2 *__restrict__ psi,
                                               const double2 *__restrict__ hpsi, int64_t ld,
                                               const double *__restrict__ eps, double *__restrict__ dots)
{
    __shared__ double red[kVecThreads / 64];
    const int band = by;
    const double e = eps[band];
    const double2 *x = psi + band * ld, *hx = hpsi + band * ld;
    double s = 0.0;
    const int64_t g0 = (int64_t)bx * kVecChunk;
    const int64_t g1 = g0 + kVecChunk < ng ? g0 + kVecChunk : ng;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kVecThreads) {
        const double2 v = x[g], hv = hx[g];
        const double dx = hv.x - e * v.x, dy = hv.y - e * v.y;
        s += dx * dx + dy * dy;
    }
    s = block_sum<kVecThreads>(s, red);
    if (threadIdx.x == 0) dots[(size_t)band * kMaxParts + bx] = s;
}
__global__ void __launch_bounds__(kVecThreads)
k_res_parts(int64_t ng, const double2 *__restrict__ psi, const double2 *__restrict__ hpsi, int64_t ld,
            const double *__restrict__ eps, double *__restrict__ dots)
{
    res_parts_body(blockIdx.x, blockIdx.y, ng, psi, hpsi, ld, eps, dots);
}
__global__ void __launch_bounds__(kVecThreads) k_res_parts_grp(GroupTab t)
{
    int e, bx, by;
    group_block(t, e, bx, by);
    const ResPartsArgs &a = *static_cast<const ResPartsArgs *>(t.args[e]);
    res_parts_body(bx, by, a.ng, a.psi, a.hpsi, a.ld, a.eps, a.dots);
}

__global__ void k_res_final(int nb, int nparts, const double *__restrict__ dots, double *__restrict__ res)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) res[b] = sqrt(sum_parts(dots + (size_t)b * kMaxParts, nparts));
}
// 256 threads per work-group, bands b = 256 bx + thread
__global__ void __launch_bounds__(256) k_res_final_grp(GroupTab t)
{
    int e, bx, by;
    group_block(t, e, bx, by);
    const ResFinalArgs &a = *static_cast<const ResFinalArgs *>(t.args[e]);
    const int b = bx * 256 + threadIdx.x;
    if (b < a.nb) a.res[b] = sqrt(sum_parts(a.dots + (size_t)b * kMaxParts, a.nparts));
}

// partial sums of |e|^2
__global__ void __launch_bounds__(kVecThreads)
k_norm_parts(int64_t ng, const double2 *__restrict__ e, int64_t lde, double *__restrict__ dots)
{
    __shared__ double red[kVecThreads / 64];
    const int band = blockIdx.y;
    const double2 *ee = e + band * lde;
    double s = 0.0;
    const int64_t g0 = (int64_t)blockIdx.x * kVecChunk;
    const int64_t g1 = g0 + kVecChunk < ng ? g0 + kVecChunk : ng;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kVecThreads) {
        const double2 d = ee[g];
        s += d.x * d.x + d.y * d.y;
    }
    s = block_sum<kVecThreads>(s, red);
    if (threadIdx.x == 0) dots[(size_t)band * kMaxParts + blockIdx.x] = s;
}

__global__ void __launch_bounds__(kVecThreads)
k_norm_scale(int64_t ng, int nparts, double2 *__restrict__ e, int64_t lde, const double *__restrict__ dots)
{
    const int band = blockIdx.y;
    const double n2 = sum_parts(dots + (size_t)band * kMaxParts, nparts);
    const double s = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
    double2 *ee = e + band * lde;
    const int64_t g0 = (int64_t)blockIdx.x * kVecChunk;
    const int64_t g1 = g0 + kVecChunk < ng ? g0 + kVecChunk : ng;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kVecThreads) {
        const double2 d = ee[g];
        ee[g] = make_double2(d.x * s, d.y * s);
    }
}

__global__ void __launch_bounds__(kVecThreads)
k_copy_bands(int64_t ng, const double2 *__restrict__ src, int64_t lds, double2 *__restrict__ dst, int64_t ldd)
{
    const int band = blockIdx.y;
    const int64_t g0 = (int64_t)blockIdx.x * kVecChunk;
    const int64_t g1 = g0 + kVecChunk < ng ? g0 + kVecChunk : ng;
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kVecThreads) dst[band * ldd + g] = src[band * lds + g];
}

inline unsigned nchunks(int64_t ng) { return (unsigned)((ng + kVecChunk - 1) / kVecChunk); }

}  // namespace

hipError_t launch_project_out(const Plan &pl, const Workspace &w, int nb, const double2 *psi, int64_t ld,
                              double2 *x)
{
    const unsigned nc = nchunks(pl.ng);
    hipLaunchKernelGGL(k_proj_parts, dim3(nc, nb), dim3(kVecThreads), 0, pl.stream, pl.ng, psi, ld, x, pl.ldv, w.dots,
                       nb);
    hipLaunchKernelGGL(k_proj_sub, dim3(nc, nb), dim3(kVecThreads), 0, pl.stream, pl.ng, (int)nc, psi, ld, x, pl.ldv,
                       w.dots, nb, pl.kin, w.sc, (double2 *)nullptr, (const double2 *)nullptr, (double *)nullptr);
    return hipGetLastError();
}

// z <- z - psi (psi^H z) / |psi|^2 with the partial r^H z of the projected z
static void project_z(const Plan &pl, const Workspace &w, int nb, const double2 *psi, int64_t ld, unsigned nc)
{
    hipLaunchKernelGGL(k_proj_parts, dim3(nc, nb), dim3(kVecThreads), 0, pl.stream, pl.ng, psi, ld, w.z, pl.ldv,
                       w.dots, nb);
    hipLaunchKernelGGL(k_proj_sub, dim3(nc, nb), dim3(kVecThreads), 0, pl.stream, pl.ng, (int)nc, psi, ld, w.z,
                       pl.ldv, w.dots, nb, pl.kin, w.sc, (double2 *)nullptr, (const double2 *)w.r,
                       w.dots + (size_t)DOT_RZ * nb * kMaxParts);
}

hipError_t launch_pcg_init(const Plan &pl, const Workspace &w, int nb, const double2 *psi, const double2 *hpsi,
                           int64_t ld, const double *eps, double2 *u, int64_t ldu, int32_t *band_flags,
                           bool correction, const double2 *proj_psi)
{
    const unsigned nc = nchunks(pl.ng);
    hipLaunchKernelGGL(k_pcg_init_parts, dim3(nc, nb), dim3(kVecThreads), 0, pl.stream, pl.ng, psi, ld, pl.kin,
                       w.dots, nb);
    hipLaunchKernelGGL((k_pcg_init<double2, double2>), dim3(nc, nb), dim3(kVecThreads), 0, pl.stream, pl.ng, (int)nc,
                       psi, hpsi, ld, eps, pl.kin, u, ldu, w.r, w.z, pl.ldv, w.dots, w.sc, nb,
                       (correction || proj_psi) ? 1 : 0);
    if (proj_psi) {
        // r0 <- (I - P) r0, z0 = K r0, z0 <- (I - P) z0, partial r0^H z0
        hipLaunchKernelGGL(k_proj_parts, dim3(nc, nb), dim3(kVecThreads), 0, pl.stream, pl.ng, proj_psi, ld, w.r,
                           pl.ldv, w.dots, nb);
        hipLaunchKernelGGL(k_proj_sub, dim3(nc, nb), dim3(kVecThreads), 0, pl.stream, pl.ng, (int)nc, proj_psi, ld,
                           w.r, pl.ldv, w.dots, nb, pl.kin, w.sc, w.z, (const double2 *)nullptr, (double *)nullptr);
        project_z(pl, w, nb, proj_psi, ld, nc);
    }
    hipLaunchKernelGGL(k_pcg_scalars, dim3(1), dim3(kVecThreads), 0, pl.stream, nb, 0, (int)nc, 0,
                       (const double *)nullptr, w.dots + (size_t)DOT_RZ * nb * kMaxParts, w.sc, w.iflags,
                       w.iflags + nb, band_flags, pl.status);
    return hipGetLastError();
}

hipError_t launch_pcg_update(const Plan &pl, const Workspace &w, int nb, double2 *u, int64_t ldu, int npq,
                             int32_t *band_flags, const double2 *proj_psi, int64_t ldpsi)
{
    const unsigned nc = nchunks(pl.ng);
    prof_mark(PARO_K_PCG_UPDATE, pl.stream, true);
    hipLaunchKernelGGL((k_pcg_update<double2, double2>), dim3(nc, nb), dim3(kVecThreads), 0, pl.stream, pl.ng, npq,
                       w.p, w.q, pl.ldv, u, ldu, w.r, w.z, pl.kin, w.dots + (size_t)DOT_PQ * nb * kMaxParts,
                       w.dots + (size_t)DOT_RZ * nb * kMaxParts, w.sc, w.iflags, nb);
    prof_mark(PARO_K_PCG_UPDATE, pl.stream, false);
    if (proj_psi) project_z(pl, w, nb, proj_psi, ldpsi, nc);
    hipLaunchKernelGGL(k_pcg_scalars, dim3(1), dim3(kVecThreads), 0, pl.stream, nb, 1, (int)nc, npq,
                       w.dots + (size_t)DOT_PQ * nb * kMaxParts, w.dots + (size_t)DOT_RZ * nb * kMaxParts, w.sc,
                       w.iflags, w.iflags + nb, band_flags, pl.status);
    return hipGetLastError();
}

hipError_t launch_pcg_init_mixed(const Plan &pl, const Workspace &w, int nb, const double2 *psi,
                                 const double2 *hpsi, int64_t ld, const double *eps, int32_t *band_flags)
{
    const unsigned nc = nchunks(pl.ng);
    hipLaunchKernelGGL(k_pcg_init_parts, dim3(nc, nb), dim3(kVecThreads), 0, pl.stream, pl.ng, psi, ld, pl.kin,
                       w.dots, nb);
    hipLaunchKernelGGL((k_pcg_init<float2, float2>), dim3(nc, nb), dim3(kVecThreads), 0, pl.stream, pl.ng, (int)nc,
                       psi, hpsi, ld, eps, pl.kin, w.d32, pl.ldv, w.r32, w.z32, pl.ldv, w.dots, w.sc, nb, 1);
    hipLaunchKernelGGL(k_pcg_scalars, dim3(1), dim3(kVecThreads), 0, pl.stream, nb, 0, (int)nc, 0,
                       (const double *)nullptr, w.dots + (size_t)DOT_RZ * nb * kMaxParts, w.sc, w.iflags,
                       w.iflags + nb, band_flags, pl.status);
    return hipGetLastError();
}

hipError_t launch_pcg_update_mixed(const Plan &pl, const Workspace &w, int nb, int npq, int32_t *band_flags)
{
    const unsigned nc = nchunks(pl.ng);
    prof_mark(PARO_K_PCG_UPDATE, pl.stream, true);
    hipLaunchKernelGGL((k_pcg_update<float2, float2>), dim3(nc, nb), dim3(kVecThreads), 0, pl.stream, pl.ng, npq,
                       w.p32, w.q32, pl.ldv, w.d32, pl.ldv, w.r32, w.z32, pl.kin,
                       w.dots + (size_t)DOT_PQ * nb * kMaxParts, w.dots + (size_t)DOT_RZ * nb * kMaxParts, w.sc,
                       w.iflags, nb);
    prof_mark(PARO_K_PCG_UPDATE, pl.stream, false);
    hipLaunchKernelGGL(k_pcg_scalars, dim3(1), dim3(kVecThreads), 0, pl.stream, nb, 1, (int)nc, npq,
                       w.dots + (size_t)DOT_PQ * nb * kMaxParts, w.dots + (size_t)DOT_RZ * nb * kMaxParts, w.sc,
                       w.iflags, w.iflags + nb, band_flags, pl.status);
    return hipGetLastError();
}

hipError_t launch_finish_correction(const Plan &pl, const Workspace &w, int nb, const double2 *base, int64_t ld,
                                    double2 *u, int64_t ldu)
{
    hipLaunchKernelGGL(k_finish_correction, dim3(nchunks(pl.ng), nb), dim3(kVecThreads), 0, pl.stream, pl.ng, base,
                       ld, w.d32, pl.ldv, u, ldu);
    return hipGetLastError();
}

hipError_t launch_residuals(const Plan &pl, const Workspace &w, int nb, const double2 *psi, const double2 *hpsi,
                            int64_t ld, const double *eps, double *res)
{
    const unsigned nc = nchunks(pl.ng);
    double *dots = w.dots + (size_t)DOT_RES * nb * kMaxParts;
    hipLaunchKernelGGL(k_res_parts, dim3(nc, nb), dim3(kVecThreads), 0, pl.stream, pl.ng, psi, hpsi, ld, eps, dots);
    hipLaunchKernelGGL(k_res_final, dim3((nb + 255) / 256), dim3(256), 0, pl.stream, nb, (int)nc, dots, res);
    return hipGetLastError();
}

hipError_t launch_normalize_bands(const Plan &pl, const Workspace &w, int nb, double2 *e, int64_t lde)
{
    const unsigned nc = nchunks(pl.ng);
    double *dots = w.dots + (size_t)DOT_RES * nb * kMaxParts;
    hipLaunchKernelGGL(k_norm_parts, dim3(nc, nb), dim3(kVecThreads), 0, pl.stream, pl.ng, e, lde, dots);
    hipLaunchKernelGGL(k_norm_scale, dim3(nc, nb), dim3(kVecThreads), 0, pl.stream, pl.ng, (int)nc, e, lde, dots);
    return hipGetLastError();
}

hipError_t launch_copy_bands(hipStream_t s, int nb, int64_t ng, const double2 *src, int64_t lds, double2 *dst,
                             int64_t ldd)
{
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_bands, dim3(nchunks(ng), nb), dim3(kVecThreads), 0, s, ng, src, lds, dst, ldd);
    return hipGetLastError();
}

}  // namespace paro

namespace paro {

// ---------------------------------------------------------------- grouped launches
// The PCG kernels of the source solve for many cells at once: the
// arguments each cell's own launches take (launch_pcg_init and
// launch_pcg_update without projection, or their mixed-precision forms),
// in its descriptor.
static void describe_pcg_common(const Plan &pl, const Workspace &w, int nb, const double2 *psi, int64_t ld,
                                int32_t *band_flags, int npq, GroupCellDesc &d)
{
    const int nc = (int)nchunks(pl.ng);
    d.iparts = PcgInitPartsArgs{psi, ld, pl.kin, w.dots, pl.ng, nb};
    d.sc0 = PcgScalarsArgs{nullptr, w.dots + (size_t)DOT_RZ * nb * kMaxParts, w.sc, w.iflags, w.iflags + nb,
                           band_flags, pl.status, nb, nc, 0};
    d.sc1 = PcgScalarsArgs{w.dots + (size_t)DOT_PQ * nb * kMaxParts, w.dots + (size_t)DOT_RZ * nb * kMaxParts, w.sc,
                           w.iflags, w.iflags + nb, band_flags, pl.status, nb, nc, npq};
}

void describe_pcg(const Plan &pl, const Workspace &w, int nb, const double2 *psi, const double2 *hpsi, int64_t ld,
                  const double *eps, double2 *u, int64_t ldu, int32_t *band_flags, bool correction, int npq,
                  GroupCellDesc &d)
{
    const int nc = (int)nchunks(pl.ng);
    describe_pcg_common(pl, w, nb, psi, ld, band_flags, npq, d);
    d.f64.init = PcgInitArgs<double2, double2>{psi, hpsi, ld, eps, pl.kin, u, ldu, w.r, w.z, pl.ldv, w.dots, w.sc,
                                               pl.ng, nc, nb, correction ? 1 : 0};
    d.f64.upd = PcgUpdateArgs<double2, double2>{w.p, w.q, pl.ldv, u, ldu, w.r, w.z, pl.kin,
                                                w.dots + (size_t)DOT_PQ * nb * kMaxParts,
                                                w.dots + (size_t)DOT_RZ * nb * kMaxParts, w.sc, w.iflags, pl.ng, npq,
                                                nb};
}

void describe_pcg_mixed(const Plan &pl, const Workspace &w, int nb, const double2 *psi, const double2 *hpsi,
                        int64_t ld, const double *eps, int32_t *band_flags, int npq, GroupCellDesc &d)
{
    const int nc = (int)nchunks(pl.ng);
    describe_pcg_common(pl, w, nb, psi, ld, band_flags, npq, d);
    d.f32.init = PcgInitArgs<float2, float2>{psi, hpsi, ld, eps, pl.kin, w.d32, pl.ldv, w.r32, w.z32, pl.ldv, w.dots,
                                             w.sc, pl.ng, nc, nb, 1};
    d.f32.upd = PcgUpdateArgs<float2, float2>{w.p32, w.q32, pl.ldv, w.d32, pl.ldv, w.r32, w.z32, pl.kin,
                                              w.dots + (size_t)DOT_PQ * nb * kMaxParts,
                                              w.dots + (size_t)DOT_RZ * nb * kMaxParts, w.sc, w.iflags, pl.ng, npq,
                                              nb};
}

namespace {

// entries of a (chunk x band) vector kernel; launches every kGroupMax entries
template <class F, class G>
hipError_t group_vec(const GroupCell *cells, int n, F args_of, G launch)
{
    GroupBuilder g;
    for (int i = 0; i < n; ++i) {
        const int nc = (int)nchunks(cells[i].pl->ng);
        g.add(args_of(cells[i].dev), (int64_t)nc * cells[i].nb, nc);
        if (g.full() || i == n - 1) {
            launch(g);
            g = GroupBuilder();
        }
    }
    return hipGetLastError();
}
template <class F>
void group_scalars(hipStream_t s, const GroupCell *cells, int n, F args_of, int stage)
{
    GroupBuilder g;
    for (int i = 0; i < n; ++i) {
        g.add(args_of(cells[i].dev), 1, 1);
        if (g.full() || i == n - 1) {
            hipLaunchKernelGGL(k_pcg_scalars_grp, dim3(g.t.n), dim3(kVecThreads), 0, s, g.t, stage);
            g = GroupBuilder();
        }
    }
}

}  // namespace

template <class C2> hipError_t launch_pcg_init_grouped(hipStream_t s, const GroupCell *cells, int n)
{
    if (n <= 0) return hipSuccess;
    hipError_t e = group_vec(cells, n, [](const GroupCellDesc *d) { return (const void *)&d->iparts; },
                             [&](const GroupBuilder &g) {
                                 hipLaunchKernelGGL(k_pcg_init_parts_grp, dim3((unsigned)g.total), dim3(kVecThreads),
                                                    0, s, g.t);
                             });
    if (e != hipSuccess) return e;
    e = group_vec(cells, n, [](const GroupCellDesc *d) { return (const void *)&group_solve_args<C2>(d)->init; },
                  [&](const GroupBuilder &g) {
                      hipLaunchKernelGGL((k_pcg_init_grp<C2, C2>), dim3((unsigned)g.total), dim3(kVecThreads), 0, s,
                                         g.t);
                  });
    if (e != hipSuccess) return e;
    group_scalars(s, cells, n, [](const GroupCellDesc *d) { return (const void *)&d->sc0; }, 0);
    return hipGetLastError();
}

template <class C2> hipError_t launch_pcg_update_grouped(hipStream_t s, const GroupCell *cells, int n)
{
    if (n <= 0) return hipSuccess;
    hipError_t e = group_vec(cells, n, [](const GroupCellDesc *d) { return (const void *)&group_solve_args<C2>(d)->upd; },
                             [&](const GroupBuilder &g) {
                                 hipLaunchKernelGGL((k_pcg_update_grp<C2, C2>), dim3((unsigned)g.total),
                                                    dim3(kVecThreads), 0, s, g.t);
                             });
    if (e != hipSuccess) return e;
    group_scalars(s, cells, n, [](const GroupCellDesc *d) { return (const void *)&d->sc1; }, 1);
    return hipGetLastError();
}

namespace {
constexpr int kUploadWords = 240;  // 1920 bytes of kernel arguments per launch
struct UploadChunk {
    uint64_t w[kUploadWords];
};
__global__ void __launch_bounds__(256) k_store_words(uint64_t *__restrict__ dst, UploadChunk c, int nwords)
{
    for (int i = threadIdx.x; i < nwords; i += 256) dst[i] = c.w[i];
}
}  // namespace

// Host bytes to device memory through kernel arguments: no host buffer has
// to outlive the call, and the upload can be captured into a graph.
hipError_t upload_bytes(hipStream_t s, void *dst, const void *src, size_t bytes)
{
    const size_t nw = (bytes + 7) / 8;
    const uint64_t *w = static_cast<const uint64_t *>(src);
    uint64_t *d = static_cast<uint64_t *>(dst);
    for (size_t o = 0; o < nw; o += kUploadWords) {
        UploadChunk c{};
        const int k = (int)std::min<size_t>(kUploadWords, nw - o);
        std::memcpy(c.w, w + o, (bytes - o * 8 < (size_t)k * 8) ? bytes - o * 8 : (size_t)k * 8);
        hipLaunchKernelGGL(k_store_words, dim3(1), dim3(256), 0, s, d + o, c, k);
    }
    return hipGetLastError();
}

void describe_residuals(const Plan &pl, const Workspace &w, int nb, const double2 *psi, const double2 *hpsi,
                        int64_t ld, const double *eps, double *res, GroupFinishArgs &f)
{
    double *dots = w.dots + (size_t)DOT_RES * nb * kMaxParts;
    f.rparts = ResPartsArgs{psi, hpsi, ld, eps, dots, pl.ng};
    f.rfinal = ResFinalArgs{dots, res, nb, (int)nchunks(pl.ng)};
}

hipError_t launch_residuals_grouped(hipStream_t s, const GroupCell *cells, int n)
{
    if (n <= 0) return hipSuccess;
    hipError_t e = group_vec(cells, n, [](const GroupCellDesc *d) { return (const void *)&d->fin.rparts; },
                             [&](const GroupBuilder &g) {
                                 hipLaunchKernelGGL(k_res_parts_grp, dim3((unsigned)g.total), dim3(kVecThreads), 0,
                                                    s, g.t);
                             });
    if (e != hipSuccess) return e;
    GroupBuilder g;
    for (int i = 0; i < n; ++i) {
        const int nbk = (cells[i].nb + 255) / 256;
        g.add(&cells[i].dev->fin.rfinal, nbk, nbk);
        if (g.full() || i == n - 1) {
            hipLaunchKernelGGL(k_res_final_grp, dim3((unsigned)g.total), dim3(256), 0, s, g.t);
            g = GroupBuilder();
        }
    }
    return hipGetLastError();
}

template hipError_t launch_pcg_init_grouped<double2>(hipStream_t, const GroupCell *, int);
template hipError_t launch_pcg_init_grouped<float2>(hipStream_t, const GroupCell *, int);
template hipError_t launch_pcg_update_grouped<double2>(hipStream_t, const GroupCell *, int);
template hipError_t launch_pcg_update_grouped<float2>(hipStream_t, const GroupCell *, int);

}  // namespace paro
