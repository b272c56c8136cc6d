// Host side of libparo: problem validation, plan construction, workspace
// layout and the C ABI entry points declared in paro.h.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "paro_internal.h"

namespace paro {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

struct Profiler {
    int kernel = 0, cap = 0, used = 0, every = 1, device = 0;
    int64_t seen = 0;  // launches of the class since the start
    bool skip = false;
    std::vector<hipEvent_t> ev;
};
static Profiler *g_prof = nullptr;
// Timing events kept per device between profiles: creating thousands of
// events takes long enough on the host for the GPU to idle and drop its
// clocks before the timed work starts.
static std::map<int, std::vector<hipEvent_t>> g_event_pool;

void prof_mark(int kernel, hipStream_t s, bool begin)
{
    Profiler *p = g_prof;
    if (!p || p->kernel != kernel) return;
    if (begin) {
        p->skip = p->used >= p->cap || (p->seen++ % p->every) != 0;
        if (!p->skip) (void)hipEventRecord(p->ev[2 * p->used], s);
    } else if (!p->skip) {
        (void)hipEventRecord(p->ev[2 * p->used + 1], s);
        ++p->used;
    }
}

static int32_t fail(int32_t code, const std::string &msg)
{
    set_error(msg);
    return code;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// reciprocal lattice b_i . a_j = 2 pi delta_ij; returns |det A|
static double reciprocal(const double *a, double *b)
{
    const double c0 = a[4] * a[8] - a[5] * a[7], c1 = a[5] * a[6] - a[3] * a[8], c2 = a[3] * a[7] - a[4] * a[6];
    const double c3 = a[7] * a[2] - a[8] * a[1], c4 = a[8] * a[0] - a[6] * a[2], c5 = a[6] * a[1] - a[7] * a[0];
    const double c6 = a[1] * a[5] - a[2] * a[4], c7 = a[2] * a[3] - a[0] * a[5], c8 = a[0] * a[4] - a[1] * a[3];
    const double det = a[0] * c0 + a[1] * c1 + a[2] * c2;
    const double tp = 6.283185307179586476925286766559 / det;
    const double c[9] = {c0, c1, c2, c3, c4, c5, c6, c7, c8};
    for (int i = 0; i < 9; ++i) b[i] = c[i] * tp;
    return std::fabs(det);
}

static double half_g2(const double *b, int n1, int n2, int n3)
{
    const double g0 = n1 * b[0] + n2 * b[3] + n3 * b[6];
    const double g1 = n1 * b[1] + n2 * b[4] + n3 * b[7];
    const double g2 = n1 * b[2] + n2 * b[5] + n3 * b[8];
    return 0.5 * (g0 * g0 + g1 * g1 + g2 * g2);
}

// Enumerate the cutoff sphere in lexicographic (n1, n2, n3) order.
static int64_t enumerate(const double *cell, double ecut, std::vector<int32_t> *out, int32_t nmax[3])
{
    double b[9];
    reciprocal(cell, b);
    const double gmax = std::sqrt(2.0 * ecut);
    int box[3];
    for (int d = 0; d < 3; ++d) {
        const double len = std::sqrt(cell[3 * d] * cell[3 * d] + cell[3 * d + 1] * cell[3 * d + 1] +
                                     cell[3 * d + 2] * cell[3 * d + 2]);
        box[d] = (int)std::floor(gmax * len / 6.283185307179586476925286766559) + 1;
    }
    int64_t n = 0;
    nmax[0] = nmax[1] = nmax[2] = 0;
    const double lim = ecut * (1.0 + 1e-12);
    for (int n1 = -box[0]; n1 <= box[0]; ++n1)
        for (int n2 = -box[1]; n2 <= box[1]; ++n2)
            for (int n3 = -box[2]; n3 <= box[2]; ++n3) {
                if (half_g2(b, n1, n2, n3) > lim) continue;
                if (out) {
                    out->push_back(n1);
                    out->push_back(n2);
                    out->push_back(n3);
                }
                ++n;
                nmax[0] = std::max(nmax[0], std::abs(n1));
                nmax[1] = std::max(nmax[1], std::abs(n2));
                nmax[2] = std::max(nmax[2], std::abs(n3));
            }
    return n;
}

static bool good_size(int n)
{
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    return n == 1 || n == 3 || n == 5;
}

// Layout of the device plan buffer.
struct PlanLayout {
    size_t kin, pt_sz, st_start, cols, vplane, tw[3], beta, dkb, miller, pcen, plm, pwid, status;
    size_t vplane32, tw32[3], beta32, bs_hi, bs_lo, bt_hi, bt_lo, total;
};

struct HostGeom {
    int64_t ng;
    int32_t nmax[3];
    int32_t nst;                  // sticks, fillers included
    int64_t ldv;
    std::vector<int32_t> cols;    // per n1 column: first stick, lowest n2, stick count
};

static PlanLayout layout(const paro_problem &p, const HostGeom &g)
{
    PlanLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t nv = (size_t)p.grid[0] * p.grid[1] * p.grid[2];
    L.kin = take(sizeof(double) * g.ng);
    L.pt_sz = take(sizeof(int32_t) * g.ng);
    L.st_start = take(sizeof(int32_t) * (g.nst + 1));
    L.cols = take(sizeof(int32_t) * g.cols.size());
    L.vplane = take(sizeof(double) * nv);
    for (int d = 0; d < 3; ++d) L.tw[d] = take(sizeof(double2) * p.grid[d]);
    L.beta = take(sizeof(double2) * (size_t)p.n_proj * g.ldv);
    L.dkb = take(sizeof(double) * std::max(1, p.n_proj));
    L.miller = take(sizeof(int32_t) * 3 * g.ng);
    L.pcen = take(sizeof(double) * 3 * std::max(1, p.n_proj));
    L.plm = take(sizeof(int32_t) * 2 * std::max(1, p.n_proj));
    L.pwid = take(sizeof(double) * std::max(1, p.n_proj));
    L.status = take(sizeof(int32_t) * 64);
    L.vplane32 = take(sizeof(float) * nv);
    for (int d = 0; d < 3; ++d) L.tw32[d] = take(sizeof(float2) * p.grid[d]);
    L.beta32 = take(sizeof(float2) * (size_t)p.n_proj * g.ldv);
    // BF16 hi / lo pairs of the projectors (split-BF16 products)
    const size_t nbs = p.n_proj > 0 ? (size_t)p.n_proj * bf16_ldk(g.ng) : 0;
    const size_t nbt = p.n_proj > 0 ? (size_t)g.ng * bf16_ldp(p.n_proj) : 0;
    L.bs_hi = take(sizeof(uint32_t) * nbs);
    L.bs_lo = take(sizeof(uint32_t) * nbs);
    L.bt_hi = take(sizeof(uint32_t) * nbt);
    L.bt_lo = take(sizeof(uint32_t) * nbt);
    L.total = off;
    return L;
}

// Validate the problem; fills the geometry.
static int32_t validate(const paro_problem *p, HostGeom *g)
{
    if (!p) return fail(PARO_EINVAL, "problem is NULL");
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(p->cell[i])) return fail(PARO_EINVAL, "cell has a non-finite entry");
    double b[9];
    const double vol = reciprocal(p->cell, b);
    if (!(vol > 0.0) || !std::isfinite(vol)) return fail(PARO_EINVAL, "cell is singular");
    if (!(p->ecut > 0.0) || !std::isfinite(p->ecut)) return fail(PARO_EINVAL, "ecut must be positive and finite");
    if (p->n_g <= 0 || !p->miller) return fail(PARO_EINVAL, "empty or NULL Miller list");
    if (!p->vloc) return fail(PARO_EINVAL, "vloc is NULL");
    for (int d = 0; d < 3; ++d)
        if (p->grid[d] <= 0) return fail(PARO_EINVAL, "grid sizes must be positive");
    if (p->n_proj < 0 || (p->n_proj > 0 && !p->proj)) return fail(PARO_EINVAL, "bad projector list");
    for (int i = 0; i < p->n_proj; ++i) {
        const paro_projector &q = p->proj[i];
        const bool lm_ok = (q.l == 0 && q.m == 0) || (q.l == 1 && q.m >= 0 && q.m <= 2);
        if (!lm_ok) return fail(PARO_EINVAL, "projector l/m must be (0,0) or (1,0..2)");
        if (!(q.width > 0.0) || !std::isfinite(q.width) || !std::isfinite(q.d) || !std::isfinite(q.center[0]) ||
            !std::isfinite(q.center[1]) || !std::isfinite(q.center[2]))
            return fail(PARO_EINVAL, "projector has a non-finite or non-positive parameter");
    }
    std::vector<int32_t> mil;
    mil.reserve((size_t)p->n_g * 3);
    const int64_t n = enumerate(p->cell, p->ecut, &mil, g->nmax);
    if (n != p->n_g) return fail(PARO_EINVAL, "Miller list size differs from the cutoff sphere");
    if (std::memcmp(mil.data(), p->miller, sizeof(int32_t) * 3 * n) != 0)
        return fail(PARO_EINVAL, "Miller list is not the cutoff sphere in canonical order");
    for (int d = 0; d < 3; ++d)
        if (p->grid[d] < 4 * g->nmax[d] + 1) return fail(PARO_EALIAS, "FFT grid smaller than 4 nmax + 1");
    const int64_t nv = (int64_t)p->grid[0] * p->grid[1] * p->grid[2];
    for (int64_t i = 0; i < nv; ++i)
        if (!std::isfinite(p->vloc[i])) return fail(PARO_EINVAL, "vloc has a non-finite value");
    if (p->grid[0] != p->grid[1] || p->grid[1] != p->grid[2] || !fft_supported(p->grid[0]) ||
        !good_size(p->grid[0]))
        return fail(PARO_EUNSUP, "this build supports cubic FFT grids of 8, 16, 24, 32, 40, 48, 64, 80, 96 or 160 points");
    g->ng = n;
    // Sticks are numbered column by column (n1 ascending), n2 ascending
    // within a column, and every n2 between a column's lowest and highest
    // populated value gets a stick: the plane kernel addresses a column's
    // sticks as one contiguous range.  Fillers hold no sphere point and stay
    // zero through the transforms.
    const int ncol = 2 * g->nmax[0] + 1;
    std::vector<int32_t> lo(ncol, INT32_MAX), hi(ncol, INT32_MIN);
    for (int64_t i = 0; i < n; ++i) {
        const int c = p->miller[3 * i] + g->nmax[0];
        lo[c] = std::min(lo[c], p->miller[3 * i + 1]);
        hi[c] = std::max(hi[c], p->miller[3 * i + 1]);
    }
    g->cols.assign(3 * ncol, 0);
    int64_t nst = 0;
    for (int c = 0; c < ncol; ++c) {
        const int64_t cnt = hi[c] >= lo[c] ? (int64_t)hi[c] - lo[c] + 1 : 0;
        g->cols[3 * c] = (int32_t)std::min<int64_t>(nst, INT32_MAX);
        g->cols[3 * c + 1] = cnt ? lo[c] : 0;
        g->cols[3 * c + 2] = (int32_t)cnt;
        nst += cnt;
    }
    if (nst >= (1 << 23)) return fail(PARO_EUNSUP, "too many sticks");
    g->nst = (int32_t)nst;
    g->ldv = (n + 31) / 32 * 32;
    return PARO_OK;
}

// bytes of a stick buffer for passes on up to m bands: a chunk of FP64
// bands or a (larger) chunk of FP32 bands
static size_t stick_buffer_bytes(const Plan &pl, size_t m)
{
    const size_t per = std::max(sizeof(double2) * std::min<size_t>(kMaxBandsPerChunk, m),
                                sizeof(float2) * std::min<size_t>(kMaxBandsPerChunk32, m));
    return per * pl.grid[2] * pl.nst;
}

size_t workspace_bytes(const Plan &pl, int nb)
{
    const size_t m = 2 * (size_t)nb;
    const size_t np = pl.nproj;
    const size_t mm = std::max(m, np);
    size_t tot = 0;
    auto add = [&](size_t bytes) { tot = align256(tot + bytes); };
    add(stick_buffer_bytes(pl, m));                            // sticks
    if (big_grid(pl.grid[0])) add(stick_buffer_bytes(pl, m));  // sticks2
    for (int i = 0; i < 4; ++i) add(sizeof(double2) * nb * pl.ldv);  // r z p q
    add(sizeof(double2) * m * pl.ldv);                          // U
    add(sizeof(double2) * m * pl.ldv);                          // W
    add(sizeof(double2) * std::max(2 * m * m, np * np));       // gram
    const size_t part = (size_t)kPartSplits * std::max(std::max(m * m, np * m), np * np);
    add(sizeof(double2) * part);                                // split-K partials
    add(sizeof(double2) * std::max<size_t>(1, np) * m);         // P
    for (int i = 0; i < 5; ++i) add(sizeof(double2) * mm * mm);  // dense
    add(sizeof(double) * dense_real_elems((int)mm));           // dreal
    add(sizeof(double) * kScalars * m);                         // sc
    add(sizeof(double) * kDotSlots * nb * kMaxParts);          // dots
    add(sizeof(int32_t) * 2 * nb);                              // iflags
    add(sizeof(double) * (3 * m + 8));                          // misc: sig_all, res, eps_all, scalars
    add(sizeof(GroupCellDesc));                                 // grouped-launch arguments
    return tot;
}

// Density workspace: the sticks of one chunk, then one partial grid per
// band group of a chunk.
size_t density_workspace_bytes(const Plan &pl, int nb, size_t *part_off)
{
    const size_t cb = std::min<size_t>(kMaxBandsPerChunk, nb);
    const size_t ngrp = (cb + kDensityBandsPerGroup - 1) / kDensityBandsPerGroup;
    const size_t nv = (size_t)pl.grid[0] * pl.grid[1] * pl.grid[2];
    const size_t off = align256(sizeof(double2) * cb * pl.grid[2] * pl.nst);
    if (part_off) *part_off = off;
    return align256(off + sizeof(double) * ngrp * nv);
}

// Projector-gradient workspace: G_a beta_p (3 n_proj x ldv), P = B^H psi
// (n_proj x nb), S = (G beta)^H psi (3 n_proj x nb), split-K partials.
ProjGradWs proj_grad_workspace(const Plan &pl, int nb, void *ws, size_t *bytes)
{
    const size_t np = pl.nproj;
    ProjGradWs w{};
    char *base = static_cast<char *>(ws);
    size_t off = 0;
    auto take = [&](size_t b) {
        char *q = base + off;
        off = align256(off + b);
        return q;
    };
    w.gbeta = (double2 *)take(sizeof(double2) * 3 * np * pl.ldv);
    w.P = (double2 *)take(sizeof(double2) * np * nb);
    w.S = (double2 *)take(sizeof(double2) * 3 * np * nb);
    w.part_elems = (size_t)kPartSplits * 3 * np * (size_t)nb;
    w.part = (double2 *)take(sizeof(double2) * w.part_elems);
    if (bytes) *bytes = off;
    return w;
}

Workspace carve_workspace(const Plan &pl, int nb, void *ws)
{
    Workspace w{};
    const size_t m = 2 * (size_t)nb;
    const size_t np = pl.nproj;
    const size_t mm = std::max(m, np);
    char *base = static_cast<char *>(ws);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base + off;
        off = align256(off + bytes);
        return p;
    };
    w.sticks = (double2 *)take(stick_buffer_bytes(pl, m));
    w.sticks2 = big_grid(pl.grid[0]) ? (double2 *)take(stick_buffer_bytes(pl, m)) : nullptr;
    w.r = (double2 *)take(sizeof(double2) * nb * pl.ldv);
    w.z = (double2 *)take(sizeof(double2) * nb * pl.ldv);
    w.p = (double2 *)take(sizeof(double2) * nb * pl.ldv);
    w.q = (double2 *)take(sizeof(double2) * nb * pl.ldv);
    w.U = (double2 *)take(sizeof(double2) * m * pl.ldv);
    w.W = (double2 *)take(sizeof(double2) * m * pl.ldv);
    w.r32 = reinterpret_cast<float2 *>(w.r);
    w.z32 = reinterpret_cast<float2 *>(w.z);
    w.p32 = reinterpret_cast<float2 *>(w.p);
    w.q32 = reinterpret_cast<float2 *>(w.q);
    w.d32 = reinterpret_cast<float2 *>(w.W);
    w.gram = (double2 *)take(sizeof(double2) * std::max(2 * m * m, np * np));
    w.part_elems = (size_t)kPartSplits * std::max(std::max(m * m, np * m), np * np);
    w.part = (double2 *)take(sizeof(double2) * w.part_elems);
    w.P = (double2 *)take(sizeof(double2) * std::max<size_t>(1, np) * m);
    for (int i = 0; i < 5; ++i) w.dense[i] = (double2 *)take(sizeof(double2) * mm * mm);
    w.dreal_elems = dense_real_elems((int)mm);
    w.dreal = (double *)take(sizeof(double) * w.dreal_elems);
    w.sc = (double *)take(sizeof(double) * kScalars * m);
    w.dots = (double *)take(sizeof(double) * kDotSlots * nb * kMaxParts);
    w.iflags = (int32_t *)take(sizeof(int32_t) * 2 * nb);
    double *misc = (double *)take(sizeof(double) * (3 * m + 8));
    w.sig_all = misc;
    w.res = misc + m;
    w.eps_all = misc + 2 * m;
    w.scal = misc + 3 * m;
    w.desc = (GroupCellDesc *)take(sizeof(GroupCellDesc));
    return w;
}

}  // namespace paro

using namespace paro;

extern "C" {

int32_t paro_abi_version(void) { return PARO_ABI_VERSION; }

const char *paro_last_error(void) { return g_last_error.c_str(); }

int32_t paro_sphere_enumerate(const double *cell, double ecut, int64_t capacity, int32_t *miller, int64_t *n_g_out,
                              int32_t *nmax_out)
{
    if (!cell || !n_g_out) return fail(PARO_EINVAL, "cell and n_g_out must not be NULL");
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(cell[i])) return fail(PARO_EINVAL, "cell has a non-finite entry");
    double b[9];
    if (!(reciprocal(cell, b) > 0.0)) return fail(PARO_EINVAL, "cell is singular");
    if (!(ecut > 0.0) || !std::isfinite(ecut)) return fail(PARO_EINVAL, "ecut must be positive and finite");
    int32_t nmax[3];
    std::vector<int32_t> mil;
    const int64_t n = enumerate(cell, ecut, miller ? &mil : nullptr, nmax);
    *n_g_out = n;
    if (nmax_out) std::memcpy(nmax_out, nmax, sizeof(nmax));
    if (miller) {
        if (capacity < n) return fail(PARO_ESIZE, "capacity smaller than the sphere");
        std::memcpy(miller, mil.data(), sizeof(int32_t) * 3 * n);
    }
    return PARO_OK;
}

int32_t paro_grid_size(const int32_t *nmax, int32_t *grid_out)
{
    if (!nmax || !grid_out) return fail(PARO_EINVAL, "NULL argument");
    for (int d = 0; d < 3; ++d) {
        if (nmax[d] < 0) return fail(PARO_EINVAL, "nmax must be >= 0");
        int n = 4 * nmax[d] + 1;
        while (!good_size(n)) ++n;
        grid_out[d] = n;
    }
    return PARO_OK;
}

int32_t paro_plan_bytes(const paro_problem *prob, size_t *bytes)
{
    if (!bytes) return fail(PARO_EINVAL, "bytes is NULL");
    HostGeom g{};
    const int32_t rc = validate(prob, &g);
    if (rc != PARO_OK) return rc;
    *bytes = layout(*prob, g).total;
    return PARO_OK;
}

int32_t paro_plan_create(const paro_problem *prob, void *dev_buf, size_t bytes, paro_stream_t stream,
                         paro_plan *plan_out)
{
    if (!plan_out) return fail(PARO_EINVAL, "plan_out is NULL");
    *plan_out = nullptr;
    HostGeom g{};
    int32_t rc = validate(prob, &g);
    if (rc != PARO_OK) return rc;
    const PlanLayout L = layout(*prob, g);
    if (!dev_buf) return fail(PARO_EINVAL, "dev_buf is NULL");
    if (bytes < L.total) return fail(PARO_ESIZE, "plan buffer smaller than paro_plan_bytes");
    if (reinterpret_cast<uintptr_t>(dev_buf) % 256) return fail(PARO_EINVAL, "dev_buf must be 256-byte aligned");
    paro_plan_s *h = new (std::nothrow) paro_plan_s();
    if (!h) return fail(PARO_EINVAL, "out of host memory");
    Plan &pl = h->pl;
    pl.stream = static_cast<hipStream_t>(stream);
    std::memcpy(pl.cell, prob->cell, sizeof(pl.cell));
    pl.omega = reciprocal(prob->cell, pl.bvec);
    pl.ecut = prob->ecut;
    std::memcpy(pl.grid, prob->grid, sizeof(pl.grid));
    std::memcpy(pl.nmax, g.nmax, sizeof(pl.nmax));
    for (int pi = 0; pi < 2; ++pi) plane_default(pl.grid[0], pi, &pl.plane_sched[pi], &pl.plane_bands[pi]);
    pl.ng = g.ng;
    pl.ldv = g.ldv;
    pl.nst = g.nst;
    pl.nproj = prob->n_proj;
    pl.ncol = 2 * g.nmax[0] + 1;
    char *base = static_cast<char *>(dev_buf);
    pl.kin = (double *)(base + L.kin);
    pl.pt_sz = (int32_t *)(base + L.pt_sz);
    pl.st_start = (int32_t *)(base + L.st_start);
    pl.cols = (int32_t *)(base + L.cols);
    pl.vplane = (double *)(base + L.vplane);
    for (int d = 0; d < 3; ++d) pl.tw[d] = (double2 *)(base + L.tw[d]);
    pl.beta = (double2 *)(base + L.beta);
    pl.dkb = (double *)(base + L.dkb);
    pl.vplane32 = (float *)(base + L.vplane32);
    for (int d = 0; d < 3; ++d) pl.tw32[d] = (float2 *)(base + L.tw32[d]);
    pl.beta32 = (float2 *)(base + L.beta32);
    pl.bf_ldk = bf16_ldk(g.ng);
    pl.bf_ldp = bf16_ldp(pl.nproj);
    pl.bs_hi = (uint32_t *)(base + L.bs_hi);
    pl.bs_lo = (uint32_t *)(base + L.bs_lo);
    pl.bt_hi = (uint32_t *)(base + L.bt_hi);
    pl.bt_lo = (uint32_t *)(base + L.bt_lo);
    pl.status = (int32_t *)(base + L.status);
    int32_t *miller_dev = (int32_t *)(base + L.miller);
    pl.miller = miller_dev;
    double *pcen = (double *)(base + L.pcen);
    int32_t *plm = (int32_t *)(base + L.plm);
    double *pwid = (double *)(base + L.pwid);

    // host tables
    const int64_t ng = g.ng;
    const int N1 = pl.grid[0], N2 = pl.grid[1], N3 = pl.grid[2];
    std::vector<double> kin(ng);
    std::vector<int32_t> pt_sz(ng), st_start(g.nst + 1, -1);
    for (int64_t i = 0; i < ng; ++i) {
        const int32_t *n = prob->miller + 3 * i;
        const int32_t *col = g.cols.data() + 3 * (n[0] + g.nmax[0]);
        const int32_t s = col[0] + (n[1] - col[1]);
        if (st_start[s] < 0) st_start[s] = (int32_t)i;
        const int z = ((n[2] % N3) + N3) % N3;
        pt_sz[i] = (s << 8) | z;
        kin[i] = half_g2(pl.bvec, n[0], n[1], n[2]);
    }
    st_start[g.nst] = (int32_t)ng;
    for (int s = g.nst - 1; s >= 0; --s)
        if (st_start[s] < 0) st_start[s] = st_start[s + 1];  // filler: empty point range
    const size_t nv = (size_t)N1 * N2 * N3;
    std::vector<double> vpl(nv);
    double vmin = prob->vloc[0];
    for (size_t i = 0; i < nv; ++i) vmin = std::min(vmin, prob->vloc[i]);
    build_plane_potential(N1, pl.grid, prob->vloc, vpl.data());
    std::vector<float> vpl32(nv);
    build_plane_potential(N1, pl.grid, prob->vloc, vpl32.data());
    pl.vmin = vmin;
    std::vector<double2> tw[3];
    std::vector<float2> tw32[3];
    for (int d = 0; d < 3; ++d) {
        const int n = pl.grid[d];
        tw[d].resize(n);
        tw32[d].resize(n);
        for (int k = 0; k < n; ++k) {
            const long double ang = 6.283185307179586476925286766559L * (long double)k / (long double)n;
            tw[d][k] = make_double2((double)cosl(ang), (double)-sinl(ang));
            tw32[d][k] = make_float2((float)cosl(ang), (float)-sinl(ang));
        }
    }
    const int np = prob->n_proj;
    std::vector<double> cen(3 * std::max(1, np)), wid(std::max(1, np)), dk(std::max(1, np));
    std::vector<int32_t> lm(2 * std::max(1, np));
    for (int i = 0; i < np; ++i) {
        for (int d = 0; d < 3; ++d) cen[3 * i + d] = prob->proj[i].center[d];
        lm[2 * i] = prob->proj[i].l;
        lm[2 * i + 1] = prob->proj[i].m;
        wid[i] = prob->proj[i].width;
        dk[i] = prob->proj[i].d;
    }
    auto up = [&](void *dst, const void *src, size_t nbytes) {
        return hipMemcpyAsync(dst, src, nbytes, hipMemcpyHostToDevice, pl.stream);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up(pl.kin, kin.data(), sizeof(double) * ng);
    if (e == hipSuccess) e = up(pl.pt_sz, pt_sz.data(), sizeof(int32_t) * ng);
    if (e == hipSuccess) e = up(pl.st_start, st_start.data(), sizeof(int32_t) * (g.nst + 1));
    if (e == hipSuccess) e = up(pl.cols, g.cols.data(), sizeof(int32_t) * g.cols.size());
    if (e == hipSuccess) e = up(pl.vplane, vpl.data(), sizeof(double) * nv);
    for (int d = 0; d < 3 && e == hipSuccess; ++d) e = up(pl.tw[d], tw[d].data(), sizeof(double2) * pl.grid[d]);
    if (e == hipSuccess) e = up(pl.vplane32, vpl32.data(), sizeof(float) * nv);
    for (int d = 0; d < 3 && e == hipSuccess; ++d) e = up(pl.tw32[d], tw32[d].data(), sizeof(float2) * pl.grid[d]);
    if (e == hipSuccess) e = up(miller_dev, prob->miller, sizeof(int32_t) * 3 * ng);
    if (e == hipSuccess) e = up(pcen, cen.data(), sizeof(double) * cen.size());
    if (e == hipSuccess) e = up(plm, lm.data(), sizeof(int32_t) * lm.size());
    if (e == hipSuccess) e = up(pwid, wid.data(), sizeof(double) * wid.size());
    if (e == hipSuccess) e = up(pl.dkb, dk.data(), sizeof(double) * dk.size());
    if (e == hipSuccess) e = hipMemsetAsync(pl.status, 0, sizeof(int32_t) * 64, pl.stream);
    if (e == hipSuccess) e = launch_build_projectors(pl, miller_dev, pcen, plm, pwid);
    if (e == hipSuccess) e = launch_to_single(pl.stream, (int64_t)pl.nproj * pl.ldv, pl.beta, pl.beta32);
    if (e == hipSuccess) e = launch_split_beta(pl);
    if (e == hipSuccess) e = hipStreamSynchronize(pl.stream);
    if (e != hipSuccess) {
        delete h;
        return fail(PARO_EHIP, std::string("plan_create: ") + hipGetErrorString(e));
    }
    *plan_out = h;
    return PARO_OK;
}

int32_t paro_plan_destroy(paro_plan plan)
{
    delete plan;
    return PARO_OK;
}

int32_t paro_plan_set_stream(paro_plan plan, paro_stream_t stream)
{
    if (!plan) return fail(PARO_EINVAL, "plan is NULL");
    plan->pl.stream = static_cast<hipStream_t>(stream);
    return PARO_OK;
}

int32_t paro_plan_get_info(paro_plan plan, paro_plan_info *info)
{
    if (!plan || !info) return fail(PARO_EINVAL, "NULL argument");
    const Plan &pl = plan->pl;
    info->n_g = pl.ng;
    for (int d = 0; d < 3; ++d) {
        info->nmax[d] = pl.nmax[d];
        info->grid[d] = pl.grid[d];
    }
    info->n_sticks = pl.nst;
    info->n_proj = pl.nproj;
    info->omega = pl.omega;
    return PARO_OK;
}

int32_t paro_workspace_bytes(paro_plan plan, int32_t nb, size_t *bytes)
{
    if (!plan || !bytes || nb <= 0) return fail(PARO_EINVAL, "bad argument");
    *bytes = workspace_bytes(plan->pl, nb);
    return PARO_OK;
}

int32_t paro_get_kinetic(paro_plan plan, double *kin_dev)
{
    if (!plan || !kin_dev) return fail(PARO_EINVAL, "NULL argument");
    const Plan &pl = plan->pl;
    PARO_HIP_TRY(hipMemcpyAsync(kin_dev, pl.kin, sizeof(double) * pl.ng, hipMemcpyDeviceToDevice, pl.stream));
    return PARO_OK;
}

int32_t paro_get_projectors(paro_plan plan, double *beta_dev)
{
    if (!plan || !beta_dev) return fail(PARO_EINVAL, "NULL argument");
    const Plan &pl = plan->pl;
    if (pl.nproj == 0) return PARO_OK;
    PARO_HIP_TRY(hipMemcpy2DAsync(beta_dev, sizeof(double2) * pl.ng, pl.beta, sizeof(double2) * pl.ldv,
                                  sizeof(double2) * pl.ng, pl.nproj, hipMemcpyDeviceToDevice, pl.stream));
    return PARO_OK;
}

int32_t paro_profile_start_sampled(int32_t kernel, int32_t max_launches, int32_t every)
{
    if (kernel < PARO_K_STICK_INV || kernel > PARO_K_DENSITY || max_launches <= 0 || max_launches > (1 << 20) ||
        every <= 0)
        return fail(PARO_EINVAL, "paro_profile_start: bad kernel class, launch count or sampling stride");
    if (g_prof) return fail(PARO_EINVAL, "paro_profile_start: a profile is already running");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(PARO_EHIP, "paro_profile_start: hipGetDevice failed");
    Profiler *p = new (std::nothrow) Profiler();
    if (!p) return fail(PARO_EINVAL, "out of host memory");
    p->kernel = kernel;
    p->cap = max_launches;
    p->every = every;
    p->device = dev;
    std::vector<hipEvent_t> &pool = g_event_pool[dev];
    const size_t need = 2 * (size_t)max_launches;
    while (p->ev.size() < need && !pool.empty()) {
        p->ev.push_back(pool.back());
        pool.pop_back();
    }
    while (p->ev.size() < need) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) {
            pool.insert(pool.end(), p->ev.begin(), p->ev.end());
            delete p;
            return fail(PARO_EHIP, "paro_profile_start: hipEventCreate failed");
        }
        p->ev.push_back(e);
    }
    g_prof = p;
    return PARO_OK;
}

int32_t paro_profile_start(int32_t kernel, int32_t max_launches)
{
    return paro_profile_start_sampled(kernel, max_launches, 1);
}

int32_t paro_profile_stop(int32_t *launches, double *total_ms)
{
    Profiler *p = g_prof;
    if (!p) return fail(PARO_EINVAL, "paro_profile_stop: no profile running");
    g_prof = nullptr;
    double tot = 0.0;
    int32_t rc = PARO_OK;
    for (int i = 0; i < p->used; ++i) {
        float ms = 0.f;
        if (hipEventSynchronize(p->ev[2 * i + 1]) != hipSuccess ||
            hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]) != hipSuccess) {
            rc = fail(PARO_EHIP, "paro_profile_stop: event query failed");
            break;
        }
        tot += ms;
    }
    if (launches) *launches = p->used;
    if (total_ms) *total_ms = tot;
    std::vector<hipEvent_t> &pool = g_event_pool[p->device];
    pool.insert(pool.end(), p->ev.begin(), p->ev.end());
    delete p;
    return rc;
}

int32_t paro_get_status(paro_plan plan, int32_t *flags)
{
    if (!plan || !flags) return fail(PARO_EINVAL, "NULL argument");
    const Plan &pl = plan->pl;
    int32_t v = 0;
    PARO_HIP_TRY(hipMemcpyAsync(&v, pl.status, sizeof(int32_t), hipMemcpyDeviceToHost, pl.stream));
    PARO_HIP_TRY(hipStreamSynchronize(pl.stream));
    PARO_HIP_TRY(hipMemsetAsync(pl.status, 0, sizeof(int32_t), pl.stream));
    *flags = v;
    return PARO_OK;
}

}  // extern "C"
