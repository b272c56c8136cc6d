// Local part of H psi through sphere -> stick -> plane FFTs (gfx950).
//
// The orbital psi(r) = sum_G c_G exp(iG.r) of eq. (e2) lives on the sphere
// of eq. (e3).  Its coefficients are scattered into sticks (the (n1, n2)
// columns holding sphere points) and transformed along n3; each z-plane is
// transformed along n2 for the populated n1 columns only and along n1 for
// every row; the row is multiplied by the local potential and sent back the
// same way; the forward stick transform gathers the sphere, scales by
// 1/(N1 N2 N3) and adds the kinetic diagonal.  This is the stiffness matrix
// element of eq. (e5), h_mn = (1/2)|G_m|^2 delta_mn + Vt(n_m - n_n), read
// with the difference G_m - G_n and the grid quadrature of the integral.
//
// Stick buffer layout: [band][n3 mod N3][stick], so a z-plane of one band
// is contiguous for the plane kernel and the stick kernels write rows of
// consecutive sticks.
#include <type_traits>
#include <vector>

#include "fft_device.h"
#include "group.h"
#include "paro_internal.h"
#include "reduce_device.h"

namespace paro {

namespace {

template <int N> constexpr bool cfg_ok()
{
    using C = FftCfg<N>;
    return C::T * C::E == N && ListInfo<typename C::Inv>::last == ListInfo<typename C::Fwd>::first;
}

// Threads of the stick kernels: 256 (32 sticks of 8 threads at 96 points),
// 128 for 160-point FP64 sticks so that the LDS tile stays at 41 KB.
template <int N3, class C2> constexpr int stick_threads() { return N3 > 96 && sizeof(C2) == 16 ? 128 : 256; }

// Thread -> (line, thread-in-line) map: the T threads of a line are in one
// wavefront, spaced 64/T lanes apart, so that 8 consecutive lanes work on 8
// consecutive lines at the same element index.  Line strides are odd (N+1
// elements) or 1, so those 8 lanes hit 8 different LDS bank groups in every
// load and exchange, and stores of consecutive sticks are contiguous.
template <int T> __device__ __forceinline__ int line_of(int tid)
{
    return (tid >> 6) * (64 / T) + (tid & 63) % (64 / T);
}
template <int T> __device__ __forceinline__ int thread_in_line(int tid) { return (tid & 63) / (64 / T); }

// Shape of the compressed-column plane stage (plane_cc_body): threads per
// work-group, the most populated columns its LDS plane holds, row passes.
template <int N, class C2> struct CcCfg {
    static constexpr int threads = 640, maxcols = 79, passes = sizeof(C2) == 16 ? 2 : 1;  // 160 points
};
template <class C2> struct CcCfg<96, C2> {
    static constexpr int threads = 512, maxcols = 47, passes = 1;
};
constexpr int kCcMaxCols = CcCfg<160, double2>::maxcols;  // 2 nmax + 1 with 160 >= 4 nmax + 1
constexpr int kCcBands = 4;                               // bands per work-group above 96 points
// plane schedule 2 at 96 points: the compressed-column stage
template <int N, class C2, int V> constexpr bool plane_cc() { return N == 96 && V == 2; }

// threads of the plane kernel: one line slot per row, rounded up to whole
// wavefronts (the compressed-column schedule: its own work-group size)
template <int N, class C2, int V = 0> constexpr int plane_threads()
{
    if constexpr (plane_cc<N, C2, V>()) return CcCfg<N, C2>::threads;
    else return (N * PlaneSched<N, C2, V>::T + 63) / 64 * 64;
}
// Line transforms done across lanes (xlane96_inverse / xlane96_forward)
// instead of through LDS: the 96-point lines, both precisions.
template <int N, class C2> constexpr bool xlane_rows() { return N == 96 || N == 160; }
// plane schedule 1 at 96 points: the cross-lane lines with two threads per lane
template <int N, class C2, int V> constexpr bool xlane_pair() { return N == 96 && V == 1; }
// go(std::integral_constant<int, V>) for plane schedule V of N points (V < plane_nsched(N))
template <int N, class F> void with_sched(int V, F &&go)
{
    if constexpr (plane_nsched(N) > 2)
        if (V == 2) return go(std::integral_constant<int, 2>());
    if constexpr (plane_nsched(N) > 1)
        if (V == 1) return go(std::integral_constant<int, 1>());
    go(std::integral_constant<int, 0>());
}
// Plans need N >= 4 n_max + 1 on every axis, so at N = 96 every populated
// index has |n| <= 23: a line's inputs x[t + 8 m] with m = 3..8 (indices
// 24..71) are zero and those outputs are never used.  The cross-lane
// kernels neither load nor store them and run the pruned 12-point DFTs
// (xlane_kept, xlane96_inverse<true>, xlane96_forward<true>).
static_assert(4 * 24 + 1 > 96, "at 96 points every populated |n| is below 24");
constexpr bool kXlanePrune = true;
// an opaque copy of the line thread index for one cross-lane call site
__device__ __forceinline__ int opaque(int t)
{
    asm volatile("" : "+v"(t));
    return t;
}
// Cross-lane transforms by length: the pruned 96-point functions, or the
// general N = 8 E schedule (160 points, every position kept).
template <int N> __host__ __device__ constexpr int xl_index(int t, int s)
{
    return N == 96 ? xlane_index(t, s) : xlane_index_e<N / 8>(t, s);
}
// At 160 points every populated |n| is at most 39 (160 >= 4 n_max + 1), so
// x[t + 8 m] is zero for m = 5..14: the pruned 20-point DFTs.
template <int N> __device__ __forceinline__ constexpr bool xl_kept(int m)
{
    return !kXlanePrune || (N == 96 ? xlane_kept(m) : xlane_kept_e<N / 8>(m));
}
template <int N, class C2> __device__ __forceinline__ void xl_inverse(C2 (&v)[N / 8], int t, const C2 *tw)
{
    if constexpr (N == 96) xlane96_inverse<kXlanePrune>(v, t, tw);
    else xlane_inverse_n<N, kXlanePrune>(v, t, tw);
}
template <int N, class C2> __device__ __forceinline__ void xl_forward(C2 (&v)[N / 8], int t, const C2 *tw)
{
    if constexpr (N == 96) xlane96_forward<kXlanePrune>(v, t, tw);
    else xlane_forward_n<N, kXlanePrune>(v, t, tw);
}
// largest populated |n| the pruned lines of N points allow
constexpr int xl_nmax_limit(int n) { return n == 96 ? 23 : n == 160 ? 39 : 1 << 30; }

// sphere points per thread whose loads the stick kernels issue together
constexpr int kGatherPts = 4;

// Sphere -> sticks, inverse transform along n3.  Line (stick) threads are
// consecutive lanes, so the exchanges between passes are wavefront-local.
// pbuf != null: PCG prologue, p <- z + beta p (first step: p <- z), the new p
// is written back and transformed.  Otherwise src is transformed as is.
template <int N3, class C2>
__device__ __forceinline__ void stick_inv_body(int bx, int by, const C2 *__restrict__ src, int64_t ld,
                                               C2 *__restrict__ pbuf, const double *__restrict__ beta, int first,
                                               C2 *__restrict__ sticks, int nst, const int32_t *__restrict__ st_start,
                                               const int32_t *__restrict__ pt_sz, const C2 *__restrict__ tw)
{
    using C = FftCfg<N3>;
    using S2 = RealOf<C2>;
    static_assert(cfg_ok<N3>(), "bad FFT config");
    constexpr int NT = stick_threads<N3, C2>();
    constexpr int T = C::T, E = C::E, S = NT / T, LD = N3 + 1;
    __shared__ C2 tile[S * LD];
    __shared__ C2 twl[N3];  // LDS copy of the twiddle table
    const int tid = threadIdx.x, sl = line_of<T>(tid), t = thread_in_line<T>(tid);
    const int s0 = bx * S, band = by;
    const int s = s0 + sl;
    const bool act = s < nst;
    for (int i = tid; i < S * LD; i += NT) tile[i] = cmk<C2>(0.0, 0.0);
    for (int i = tid; i < N3; i += NT) twl[i] = tw[i];
    __syncthreads();
    const int p0 = st_start[s0], p1 = st_start[min(s0 + S, nst)];
    const C2 *x = src + band * ld;
    C2 *pb = pbuf ? pbuf + band * ld : nullptr;
    const S2 bt = (pbuf && !first) ? (S2)beta[band] : (S2)0;
    // all loads of kGatherPts points per thread first, then the arithmetic
    // and the stores, so that one memory latency covers them (a lane past
    // the range loads point p0 and stores nothing)
    for (int base = p0 + tid; base < p1; base += kGatherPts * NT) {
        C2 xv[kGatherPts], po[kGatherPts];
        int sz[kGatherPts];
#pragma unroll
        for (int u = 0; u < kGatherPts; ++u) {
            const int idx = base + u * NT, i = idx < p1 ? idx : p0;
            xv[u] = x[i];
            sz[u] = pt_sz[i];
            if (pb && !first) po[u] = pb[i];
        }
#pragma unroll
        for (int u = 0; u < kGatherPts; ++u) {
            const int idx = base + u * NT;
            if (idx >= p1) break;
            C2 val = xv[u];
            if (pb) {
                if (!first) {
                    val.x += bt * po[u].x;
                    val.y += bt * po[u].y;
                }
                pb[idx] = val;
            }
            tile[((sz[u] >> 8) - s0) * LD + (sz[u] & 255)] = val;
        }
    }
    __syncthreads();
    C2 v[E];
    C2 *line = tile + sl * LD;
    C2 *out = sticks + (size_t)band * N3 * nst;
    if constexpr (xlane_rows<N3, C2>()) {
        // cross-lane transform (every lane takes part; the tile is zero past
        // the last stick), outputs stored in the schedule's register order
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = xl_kept<N3>(m) ? line[t + T * m] : cmk<C2>(0.0, 0.0);
        xl_inverse<N3>(v, opaque(t), twl);
        if (act) {
#pragma unroll
            for (int e = 0; e < E; ++e) out[(size_t)xl_index<N3>(t, e) * nst + s] = v[e];
        }
    } else {
        if (act) pass_load<N3, T, E, ListInfo<typename C::Inv>::first>(v, t, [&](int i) { return line[i]; });
        stockham<N3, +1, true>(typename C::Inv{}, v, t, act, line, 1, twl);
        if (act)
            final_foreach<N3, T, E, ListInfo<typename C::Inv>::last>(
                v, t, [&](int i, int e) { out[(size_t)i * nst + s] = v[e]; });
    }
}
template <int N3, class C2>
__global__ void __launch_bounds__((stick_threads<N3, C2>()))
k_stick_inv(const C2 *__restrict__ src, int64_t ld, C2 *__restrict__ pbuf, const double *__restrict__ beta, int first,
            C2 *__restrict__ sticks, int nst, const int32_t *__restrict__ st_start, const int32_t *__restrict__ pt_sz,
            const C2 *__restrict__ tw)
{
    stick_inv_body<N3, C2>(blockIdx.x, blockIdx.y, src, ld, pbuf, beta, first, sticks, nst, st_start, pt_sz, tw);
}
template <int N3, class C2>
__global__ void __launch_bounds__((stick_threads<N3, C2>())) k_stick_inv_grp(GroupTab t, int first)
{
    int e, bx, by;
    group_block(t, e, bx, by);
    const StickInvArgs<C2> &a = *static_cast<const StickInvArgs<C2> *>(t.args[e]);
    stick_inv_body<N3, C2>(bx, by, a.src, a.ld, a.pbuf, a.beta, first, a.sticks, a.nst, a.st_start, a.pt_sz, a.tw);
}


// ---------------------------------------------------------------- compressed-column plane stage
// One z-plane of up to bpg bands per work-group, with the plane held in LDS
// in compressed-column form: plane[c][y] for the populated columns
// c = n1 + nmax1 only (ncol <= CcCfg::maxcols), y = n2 mod N.  Per band:
// the inverse column transforms (sticks -> plane), the row transforms
// (inverse, x V, forward; populated entries read and written back), the
// forward column transforms (plane -> sticks).  All lines are cross-lane
// transforms (8 lanes, no exchange space), so LDS holds only the plane.
// Above 96 points (k_plane_cc): FP32 holds the whole plane, 79 x 161 x 8 B
// = 102 KB at most.  FP64 would need twice that, so the rows go in two
// passes of N/2 (y < N/2, then y >= N/2): each pass stores half of every
// inverse column's outputs, and the forward columns, linear in their
// input, add the second pass's transform of the other half to the stick
// values the first pass wrote.  The outputs go to a second stick buffer
// (sout): the second pass reads its inputs again from sin.  At 96 points
// (plane schedule 2): one pass, 47 x 97 x 16 B = 73 KB in FP64, so two
// 512-thread work-groups share a compute unit, and the outputs go back in
// place (sout = sin: every stick entry is read and written by the same
// line slot, the writes after a barrier that follows the reads).
// Wavefronts whose line slots hold no populated column skip the column
// transforms; the swaps inside a transform pair lanes of one line, and
// every skip is uniform over a wavefront.

template <int N, class C2>
__device__ __forceinline__ void plane_cc_body(int z, int by, int bpg, const C2 *sin, C2 *sout, int nst, int N3, int nb,
                                              const int32_t *__restrict__ cols, int ncol, int nmax1,
                                              const RealOf<C2> *__restrict__ vperm, const C2 *__restrict__ tw)
{
    static_assert(xlane_rows<N, C2>(), "cross-lane lines");
    using CC = CcCfg<N, C2>;
    constexpr int T = 8, E = N / 8, NP = CC::passes, NR = N / NP, LDY = NR + 1;
    constexpr int SLOTS = CC::threads / T, WS = 64 / T;  // line slots per work-group and per wavefront
    // one line slot per column; the last row round ends on a wavefront boundary
    static_assert(SLOTS >= CC::maxcols && (NR % SLOTS) % WS == 0, "cc plane shape");
    __shared__ C2 plane[CC::maxcols * LDY];
    __shared__ C2 twl[N];
    const int tid = threadIdx.x, sl = line_of<T>(tid), t = thread_in_line<T>(tid);
    for (int i = tid; i < N; i += CC::threads) twl[i] = tw[i];
    __syncthreads();
    const int b0 = by * bpg, b1 = min(b0 + bpg, nb);
    const int c = sl;
    const bool colact = c < ncol;
    const bool wave_cols = (tid >> 6) * WS < ncol;  // this wavefront holds a populated column
    int cst = 0, ylo = 0, cnt = 0;
    if (colact) {
        cst = cols[3 * c];
        ylo = cols[3 * c + 1];
        cnt = cols[3 * c + 2];
    }
    for (int k = b0; k < b1; ++k) {
#pragma unroll 1
        for (int p = 0; p < NP; ++p) {
            C2 v[E];
            if (wave_cols) {
                // inverse along n2 of column c; keep the outputs of this pass's rows.
                // (The index values of each stage are made opaque, so that the
                // compiler recomputes them per stage instead of holding every
                // stage's offsets in registers across the band loop.)
                int tt = t, lo = ylo, n = cnt;
                asm volatile("" : "+v"(tt), "+v"(lo), "+v"(n));
                const C2 *tz = sin + ((size_t)k * N3 + z) * nst + cst;
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int i = tt + T * m;
                    const int q = (i > N / 2 ? i - N : i) - lo;
                    v[m] = (xl_kept<N>(m) && colact && (unsigned)q < (unsigned)n) ? tz[q] : cmk<C2>(0.0, 0.0);
                }
                xl_inverse<N>(v, opaque(t), twl);
                if (colact) {
                    C2 *pc = plane + c * LDY;
                    const int ts = opaque(t);
#pragma unroll
                    for (int s = 0; s < E; ++s) {
                        const int y = xl_index<N>(ts, s);
                        if (NP == 1 || y / NR == p) pc[y - p * NR] = v[s];
                    }
                }
            }
            __syncthreads();
#pragma unroll 1
            for (int r = sl; r < NR; r += SLOTS) {
                // row y = p NR + r along n1: inverse, x V, forward (populated columns only)
                const int y = p * NR + r;
                int tt = t, nm = nmax1;
                asm volatile("" : "+v"(tt), "+v"(nm));
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int i = tt + T * m;
                    const bool pop = xl_kept<N>(m) && (i <= nm || i >= N - nm);
                    v[m] = pop ? plane[(i <= nm ? i + nm : i - N + nm) * LDY + r] : cmk<C2>(0.0, 0.0);
                }
                xl_inverse<N>(v, opaque(t), twl);
                const RealOf<C2> *vp = vperm + (((size_t)z * N + y) * T + opaque(t)) * E;
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] = cscale(v[e], vp[e]);
                xl_forward<N>(v, opaque(t), twl);
                int tw2 = t, nm2 = nmax1;
                asm volatile("" : "+v"(tw2), "+v"(nm2));
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int i = tw2 + T * m;
                    if (xl_kept<N>(m) && (i <= nm2 || i >= N - nm2))
                        plane[(i <= nm2 ? i + nm2 : i - N + nm2) * LDY + r] = v[m];
                }
            }
            __syncthreads();
            if (wave_cols) {
                // forward along n2 of column c from this pass's rows; back to the sticks
                const int ts = opaque(t);
                const C2 *pc = plane + (colact ? c : 0) * LDY;
#pragma unroll
                for (int s = 0; s < E; ++s) {
                    const int y = xl_index<N>(ts, s);
                    v[s] = (colact && (NP == 1 || y / NR == p)) ? pc[y - p * NR] : cmk<C2>(0.0, 0.0);
                }
                xl_forward<N>(v, opaque(t), twl);
                if (colact) {
                    int tt = t, lo = ylo, n = cnt;
                    asm volatile("" : "+v"(tt), "+v"(lo), "+v"(n));
                    C2 *tz = sout + ((size_t)k * N3 + z) * nst + cst;
#pragma unroll
                    for (int m = 0; m < E; ++m) {
                        const int i = tt + T * m;
                        const int q = (i > N / 2 ? i - N : i) - lo;
                        if (xl_kept<N>(m) && (unsigned)q < (unsigned)n) {
                            if (p == 0) tz[q] = v[m];
                            else tz[q] = cadd(tz[q], v[m]);
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
}
template <int N, class C2>
__global__ void __launch_bounds__((CcCfg<N, C2>::threads))
k_plane_cc(const C2 *__restrict__ sin, C2 *__restrict__ sout, int nst, int N3, int nb, const int32_t *__restrict__ cols,
           int ncol, int nmax1, const RealOf<C2> *__restrict__ vperm, const C2 *__restrict__ tw)
{
    plane_cc_body<N, C2>(blockIdx.x, blockIdx.y, kCcBands, sin, sout, nst, N3, nb, cols, ncol, nmax1, vperm, tw);
}


// One z-plane of bands b0 .. b1-1: inverse along n2 (populated n1 columns),
// along n1 (all rows), times V, forward along n1, forward along n2; in place
// in the stick buffer.  A column's sticks are one contiguous range (n2
// ascending), so the column transforms read their input from and write
// their output to the stick buffer directly; the plane in LDS only carries
// the data between the column and row stages.
//
// The populated n1 columns are |n1| <= nmax1, at most N/2 of the N, so the
// plane holds the columns of two bands at once: even bands (counted from
// b0) at x = n1 mod N, odd bands shifted by N/2.  The line slots split in
// two halves: while the lower half runs the forward column transforms of
// band k-1, the upper half runs the inverse column transforms of band k;
// then all slots run the row transforms of band k.  Two work-group barriers
// per band.  Every transform line is wavefront-local.  The potential is
// stored in the order the row threads hold their values, so each thread
// reads E consecutive doubles, which the bands of the work-group share
// through the cache.
template <int N, class C2, int V>
__device__ __forceinline__ void plane_body(int bx, int by, C2 *__restrict__ sticks, int nst, int N3, int nb,
                                           const int32_t *__restrict__ cols, const RealOf<C2> *__restrict__ vperm,
                                           int nmax1, const C2 *__restrict__ tw, int bpb)
{
    using VR = RealOf<C2>;
    using C = PlaneSched<N, C2, V>;
    static_assert(C::T * C::E == N && ListInfo<typename C::Inv>::last == ListInfo<typename C::Fwd>::first,
                  "bad plane FFT config");
    using Inv = typename C::Inv;
    using Fwd = typename C::Fwd;
    constexpr int T = C::T, E = C::E, LDX = N + 1, HALF = N / 2;
    constexpr int RL = ListInfo<Inv>::last;
    __shared__ C2 plane[N * LDX];
    __shared__ C2 twl[N];  // LDS copy of the twiddle table
    const int tid = threadIdx.x;
    const int z = bx;
    for (int i = tid; i < N; i += plane_threads<N, C2, V>()) twl[i] = tw[i];
    __syncthreads();
    const int b0 = by * bpb, b1 = min(b0 + bpb, nb);
    const int nbk = b1 - b0;
    const int ncol = 2 * nmax1 + 1;
    const int slot = line_of<T>(tid), t = thread_in_line<T>(tid);
    // column role of this line slot: lower half forward, upper half inverse
    const bool lower = slot < HALF;
    const int c = lower ? slot : slot - HALF;
    const bool colact = c < ncol && slot < N;
    int xcol = c - nmax1;
    xcol += xcol < 0 ? N : 0;
    const bool rowact = slot < N;
    C2 *row = plane + (rowact ? slot : 0) * LDX;
    int cst = 0, ylo = 0, cnt = 0;
    if (colact) {
        cst = cols[3 * c];
        ylo = cols[3 * c + 1];
        cnt = cols[3 * c + 2];
    }
    // offset of grid row i (n2 = i or i - N) in this column's stick range, or -1
    auto stick_of = [&](int i) {
        const int k = (i > N / 2 ? i - N : i) - ylo;
        return (unsigned)k < (unsigned)cnt ? k : -1;
    };
    int64_t vofs = (((int64_t)z * N + (rowact ? slot : 0)) * T + t) * E;  // this thread's potential values
    for (int k = 0; k <= nbk; ++k) {
        // Opaque per band: keeps the compiler from hoisting the potential
        // loads and the per-element stick offsets out of the band loop,
        // which would hold them in registers across all stages.
        // (The offset, not a pointer, is made opaque: the loads stay global
        // loads; a flat load would hold up the LDS waits as well.)
        asm volatile("" : "+v"(ylo), "+v"(cnt), "+v"(vofs));
        const VR *vp = vperm + vofs;
        C2 v[E];
        {
            // column phase: forward of band k-1 (lower), inverse of band k (upper)
            const int kb = lower ? k - 1 : k;
            const bool act = colact && kb >= 0 && kb < nbk;
            int xs = xcol + ((kb & 1) ? HALF : 0);
            xs -= xs >= N ? N : 0;
            C2 *col = plane + (act ? xs : 0);
            C2 *tz = sticks + ((size_t)(b0 + (act ? kb : 0)) * N3 + z) * nst + cst;
            if constexpr (xlane_pair<N, C2, V>()) {
                // as below, with the eight-lane threads 2 t and 2 t + 1 in
                // this lane (register sets a and b)
                const int ta = 2 * t, tb = ta + 1;
                if (kb >= 0 && kb < nbk) {
                    C2 va[12], vb[12];
                    if (lower) {
#pragma unroll
                        for (int e = 0; e < 12; ++e) {
                            va[e] = act ? col[xlane_index(ta, e) * LDX] : cmk<C2>(0.0, 0.0);
                            vb[e] = act ? col[xlane_index(tb, e) * LDX] : cmk<C2>(0.0, 0.0);
                        }
                        xlane96x2_forward<kXlanePrune>(va, vb, opaque(t), twl);
                        if (act) {
#pragma unroll
                            for (int m = 0; m < 12; ++m) {
                                if (!xlane_kept(m)) continue;
                                const int qa = stick_of(ta + 8 * m), qb = stick_of(tb + 8 * m);
                                if (qa >= 0) tz[qa] = va[m];
                                if (qb >= 0) tz[qb] = vb[m];
                            }
                        }
                    } else {
#pragma unroll
                        for (int m = 0; m < 12; ++m) {
                            const int qa = (act && xlane_kept(m)) ? stick_of(ta + 8 * m) : -1;
                            const int qb = (act && xlane_kept(m)) ? stick_of(tb + 8 * m) : -1;
                            va[m] = qa >= 0 ? tz[qa] : cmk<C2>(0.0, 0.0);
                            vb[m] = qb >= 0 ? tz[qb] : cmk<C2>(0.0, 0.0);
                        }
                        xlane96x2_inverse<kXlanePrune>(va, vb, opaque(t), twl);
                        if (act) {
#pragma unroll
                            for (int e = 0; e < 12; ++e) {
                                col[xlane_index(ta, e) * LDX] = va[e];
                                col[xlane_index(tb, e) * LDX] = vb[e];
                            }
                        }
                    }
                }
            } else if constexpr (xlane_rows<N, C2>()) {
                // Column transforms across lanes too.  The forward column
                // reads the plane in the register order the cross-lane
                // inverse leaves (xlane_index) and the inverse column writes
                // it in that order; the transforms run on every lane of a
                // wavefront (lines past the populated columns on zeros,
                // without loads or stores), since a swap only pairs lanes of
                // one line.
                if (kb >= 0 && kb < nbk) {
                    if (lower) {
#pragma unroll
                        for (int e = 0; e < E; ++e) v[e] = act ? col[xlane_index(t, e) * LDX] : cmk<C2>(0.0, 0.0);
                        xlane96_forward<kXlanePrune>(v, opaque(t), twl);
                        if (act) {
#pragma unroll
                            for (int m = 0; m < E; ++m) {
                                if (!xlane_kept(m)) continue;
                                const int q = stick_of(t + T * m);
                                if (q >= 0) tz[q] = v[m];
                            }
                        }
                    } else {
#pragma unroll
                        for (int m = 0; m < E; ++m) {
                            const int q = (act && xlane_kept(m)) ? stick_of(t + T * m) : -1;
                            v[m] = q >= 0 ? tz[q] : cmk<C2>(0.0, 0.0);
                        }
                        xlane96_inverse<kXlanePrune>(v, opaque(t), twl);
                        if (act) {
#pragma unroll
                            for (int e = 0; e < E; ++e) col[xlane_index(t, e) * LDX] = v[e];
                        }
                    }
                }
            } else if (lower) {
                if (act) pass_load<N, T, E, ListInfo<Fwd>::first>(v, t, [&](int i) { return col[i * LDX]; });
                stockham_c<C, -1, true>(Fwd{}, v, t, act, col, LDX, twl);
                if (act) final_foreach<N, T, E, ListInfo<Fwd>::last>(v, t, [&](int i, int e) {
                    const int q = stick_of(i);
                    if (q >= 0) tz[q] = v[e];
                });
            } else {
                if (act) pass_load<N, T, E, ListInfo<Inv>::first>(v, t, [&](int i) {
                    const int q = stick_of(i);
                    return q >= 0 ? tz[q] : cmk<C2>(0.0, 0.0);
                });
                stockham_c<C, +1, true>(Inv{}, v, t, act, col, LDX, twl);
                wave_lds_sync();
                if (act) final_foreach<N, T, E, RL>(v, t, [&](int i, int e) { col[i * LDX] = v[e]; });
            }
        }
        __syncthreads();
        if (k == nbk) break;
        // n1 rows of band k: inverse, multiply by V, forward; only the
        // populated n1 columns are read and written back.  The potential is
        // loaded first so that its latency overlaps the inverse transform.
        {
            const int sh = (k & 1) ? HALF : 0;
            auto at = [&](int i) {  // plane slot of n1 index i (populated only)
                int x = i + sh;
                return x - (x >= N ? N : 0);
            };
            if constexpr (xlane_pair<N, C2, V>()) {
                // as below, with the eight-lane threads 2 t and 2 t + 1 in
                // this lane; their potential values are this lane's 24
                static_assert(plane_threads<N, C2, V>() == N * T && T == 4 && E == 24,
                              "paired cross-lane rows: 96 x 4 lanes");
                const int ta = 2 * t, tb = ta + 1;
                C2 va[12], vb[12];
#pragma unroll
                for (int m = 0; m < 12; ++m) {
                    const int ia = ta + 8 * m, ib = tb + 8 * m;
                    va[m] = (xlane_kept(m) && (ia <= nmax1 || ia >= N - nmax1)) ? row[at(ia)] : cmk<C2>(0.0, 0.0);
                    vb[m] = (xlane_kept(m) && (ib <= nmax1 || ib >= N - nmax1)) ? row[at(ib)] : cmk<C2>(0.0, 0.0);
                }
                xlane96x2_inverse<kXlanePrune>(va, vb, opaque(t), twl);
#pragma unroll
                for (int e = 0; e < 12; ++e) {
                    va[e] = cscale(va[e], vp[e]);
                    vb[e] = cscale(vb[e], vp[12 + e]);
                }
                xlane96x2_forward<kXlanePrune>(va, vb, opaque(t), twl);
#pragma unroll
                for (int m = 0; m < 12; ++m) {
                    const int ia = ta + 8 * m, ib = tb + 8 * m;
                    if (xlane_kept(m) && (ia <= nmax1 || ia >= N - nmax1)) row[at(ia)] = va[m];
                    if (xlane_kept(m) && (ib <= nmax1 || ib >= N - nmax1)) row[at(ib)] = vb[m];
                }
            } else if constexpr (xlane_rows<N, C2>()) {
                // Thread t reads and writes the row elements t + T m only,
                // and every exchange is a lane swap: no LDS traffic besides
                // the populated entries, no wave synchronisation.  All N
                // line slots are rows here (N T threads), so every lane of
                // each wavefront takes part in the swaps.
                static_assert(plane_threads<N, C2, V>() == N * T && T == 8 && E == 12, "cross-lane rows: 96 x 8 lanes");
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int i = t + T * m;
                    v[m] = (xlane_kept(m) && (i <= nmax1 || i >= N - nmax1)) ? row[at(i)] : cmk<C2>(0.0, 0.0);
                }
                xlane96_inverse<kXlanePrune>(v, opaque(t), twl);
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] = cscale(v[e], vp[e]);
                // the forward transform rereads the twiddles rather than
                // keeping the inverse's thirteen live across the multiply
                xlane96_forward<kXlanePrune>(v, opaque(t), twl);
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int i = t + T * m;
                    if (xlane_kept(m) && (i <= nmax1 || i >= N - nmax1)) row[at(i)] = v[m];
                }
            } else {
                VR vr[E];
#pragma unroll
                for (int e = 0; e < E; ++e) vr[e] = vp[e];
                if (rowact) pass_load<N, T, E, ListInfo<Inv>::first>(v, t, [&](int i) {
                    return (i <= nmax1 || i >= N - nmax1) ? row[at(i)] : cmk<C2>(0.0, 0.0);
                });
                stockham_c<C, +1, true>(Inv{}, v, t, rowact, row, 1, twl);
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] = cscale(v[e], vr[e]);
                stockham_c<C, -1, true>(Fwd{}, v, t, rowact, row, 1, twl);
                wave_lds_sync();
                if (rowact) final_foreach<N, T, E, ListInfo<Fwd>::last>(v, t, [&](int i, int e) {
                    if (i <= nmax1 || i >= N - nmax1) row[at(i)] = v[e];
                });
            }
        }
        __syncthreads();
    }
}
template <int N, class C2, int V>
__global__ void __launch_bounds__((plane_threads<N, C2, V>()))
__attribute__((amdgpu_waves_per_eu(PlaneSched<N, C2, V>::min_waves)))
k_plane(C2 *__restrict__ sticks, int nst, int N3, int nb, const int32_t *__restrict__ cols,
        const RealOf<C2> *__restrict__ vperm, int nmax1, const C2 *__restrict__ tw, int bpb)
{
    if constexpr (plane_cc<N, C2, V>())
        plane_cc_body<N, C2>(blockIdx.x, blockIdx.y, bpb, sticks, sticks, nst, N3, nb, cols, 2 * nmax1 + 1, nmax1,
                             vperm, tw);
    else plane_body<N, C2, V>(blockIdx.x, blockIdx.y, sticks, nst, N3, nb, cols, vperm, nmax1, tw, bpb);
}
template <int N, class C2, int V>
__global__ void __launch_bounds__((plane_threads<N, C2, V>()))
__attribute__((amdgpu_waves_per_eu(PlaneSched<N, C2, V>::min_waves)))
k_plane_grp(GroupTab t)
{
    int e, bx, by;
    group_block(t, e, bx, by);
    const PlaneArgs<C2> &a = *static_cast<const PlaneArgs<C2> *>(t.args[e]);
    if constexpr (plane_cc<N, C2, V>())
        plane_cc_body<N, C2>(bx, by, a.bpb, a.sticks, a.sticks, a.nst, a.N3, a.nb, a.cols, 2 * a.nmax1 + 1, a.nmax1,
                             a.vperm, a.tw);
    else plane_body<N, C2, V>(bx, by, a.sticks, a.nst, a.N3, a.nb, a.cols, a.vperm, a.nmax1, a.tw, a.bpb);
}


// Density of bands b0 .. b1-1 (b1 - b0 <= bands per group) on one
// z-plane: inverse along n2 and n1 as in k_plane, then w_b |psi_b(r)|^2
// summed over the group's bands in registers, in band order.  With PAIR,
// two bands per step: the lower line slots run the column transforms of
// band k (at x = n1 mod N), the upper slots those of band k + 1 (shifted
// by N/2); the row stage then reads both bands' populated entries of a row
// into registers before the first row transform uses the row as exchange
// space.  Without PAIR (large N, where the second band's registers would
// spill) one band per step, its columns on the lower slots, and the
// running sums wait in LDS between row stages, in the unpopulated n1 range
// of the thread's own row (N - 2 nmax1 - 1 >= N / 2 complex slots, which
// the column stage never writes), so that they take no registers during
// the column transforms.  With the cross-lane 96-point schedule the rows
// need no exchange space and the sums stay in registers.  The group's
// partial plane is written in the row threads' register order,
// part[((z N + y) T + t) E + e].
template <int N> constexpr bool density_pairs() { return N <= 64; }

template <int N>
__global__ void __launch_bounds__((plane_threads<N, double2>()))
__attribute__((amdgpu_waves_per_eu(PlaneCfgP<N, double2>::min_waves)))
k_plane_density(const double2 *__restrict__ sticks, int nst, int N3, int nb, int bpg,
                const int32_t *__restrict__ cols, int nmax1, const double *__restrict__ weights,
                const double2 *__restrict__ tw, double *__restrict__ part)
{
    using C = PlaneCfgP<N, double2>;
    using Inv = typename C::Inv;
    constexpr int T = C::T, E = C::E, LDX = N + 1, HALF = N / 2;
    constexpr int RL = ListInfo<Inv>::last;
    __shared__ double2 plane[N * LDX];
    __shared__ double2 twl[N];  // LDS copy of the twiddle table
    const int tid = threadIdx.x;
    const int z = blockIdx.x, g = blockIdx.y;
    for (int i = tid; i < N; i += plane_threads<N, double2>()) twl[i] = tw[i];
    __syncthreads();
    const int b0 = g * bpg, b1 = min(b0 + bpg, nb);
    const int ncol = 2 * nmax1 + 1;
    const int slot = line_of<T>(tid);
    int t = thread_in_line<T>(tid);
    const bool lower = slot < HALF;
    const int c = lower ? slot : slot - HALF;
    const bool colact = c < ncol && slot < N;
    int xcol = c - nmax1;
    xcol += xcol < 0 ? N : 0;
    const bool rowact = slot < N;
    double2 *row = plane + (rowact ? slot : 0) * LDX;
    int cst = 0, ylo = 0, cnt = 0;
    if (colact) {
        cst = cols[3 * c];
        ylo = cols[3 * c + 1];
        cnt = cols[3 * c + 2];
    }
    auto stick_of = [&](int i) {
        const int k = (i > N / 2 ? i - N : i) - ylo;
        return (unsigned)k < (unsigned)cnt ? k : -1;
    };
    constexpr bool PAIR = density_pairs<N>();
    double acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = 0.0;
    // this thread's E running sums between row stages (without PAIR)
    double *stash = reinterpret_cast<double *>(row + nmax1 + 1) + t * E;
    if (!PAIR && !xlane_rows<N, double2>() && rowact)
#pragma unroll
        for (int e = 0; e < E; ++e) stash[e] = 0.0;
    for (int k = b0; k < b1; k += PAIR ? 2 : 1) {
        // Opaque per stage: keeps the per-element stick offsets and LDS
        // addresses of one stage from being hoisted out of the band loop
        // and held in registers through the other stage.
        asm volatile("" : "+v"(ylo), "+v"(cnt), "+v"(t), "+v"(xcol));
        {
            const int kb = lower ? k : (PAIR ? k + 1 : b1);
            const bool act = colact && kb < b1;
            int xs = xcol + (lower ? 0 : HALF);
            xs -= xs >= N ? N : 0;
            double2 *col = plane + (act ? xs : 0);
            const double2 *tz = sticks + ((size_t)(act ? kb : 0) * N3 + z) * nst + cst;
            double2 v[E];
            if constexpr (xlane_rows<N, double2>()) {
                // cross-lane inverse column (lower slots; the upper ones
                // have no column without PAIR), written in the register
                // order the row stage's loads expect
                if (lower) {
#pragma unroll
                    for (int m = 0; m < E; ++m) {
                        const int q = (act && xlane_kept(m)) ? stick_of(t + T * m) : -1;
                        v[m] = q >= 0 ? tz[q] : cmk<double2>(0.0, 0.0);
                    }
                    xlane96_inverse<kXlanePrune>(v, opaque(t), twl);
                    if (act) {
#pragma unroll
                        for (int e = 0; e < E; ++e) col[xlane_index(t, e) * LDX] = v[e];
                    }
                }
            } else {
                if (act) pass_load<N, T, E, ListInfo<Inv>::first>(v, t, [&](int i) {
                    const int q = stick_of(i);
                    return q >= 0 ? tz[q] : cmk<double2>(0.0, 0.0);
                });
                stockham_c<C, +1, true>(Inv{}, v, t, act, col, LDX, twl);
                wave_lds_sync();
                if (act) final_foreach<N, T, E, RL>(v, t, [&](int i, int e) { col[i * LDX] = v[e]; });
            }
        }
        __syncthreads();
        if constexpr (xlane_rows<N, double2>()) {
            // cross-lane inverse rows; the running sums stay in registers,
            // in the schedule's register order
            static_assert(!PAIR, "cross-lane density rows: one band per step");
            double2 v[E];
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int i = t + T * m;
                v[m] = (xlane_kept(m) && (i <= nmax1 || i >= N - nmax1)) ? row[i] : cmk<double2>(0.0, 0.0);
            }
            xlane96_inverse<kXlanePrune>(v, opaque(t), twl);
            const double w0 = weights ? weights[k] : 1.0;
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] += w0 * (v[e].x * v[e].x + v[e].y * v[e].y);
            __syncthreads();
            continue;
        }
        asm volatile("" : "+v"(t));
        {
            const bool two = PAIR && k + 1 < b1;
            auto populated = [&](int i) { return i <= nmax1 || i >= N - nmax1; };
            double2 v0[E], v1[E];
            if (rowact) {
                pass_load<N, T, E, ListInfo<Inv>::first>(v0, t, [&](int i) {
                    return populated(i) ? row[i] : cmk<double2>(0.0, 0.0);
                });
                if (PAIR)
                    pass_load<N, T, E, ListInfo<Inv>::first>(v1, t, [&](int i) {
                        int x = i + HALF;
                        x -= x >= N ? N : 0;
                        return (two && populated(i)) ? row[x] : cmk<double2>(0.0, 0.0);
                    });
            }
            if (!PAIR && rowact)
#pragma unroll
                for (int e = 0; e < E; ++e) acc[e] = stash[e];
            wave_lds_sync();
            stockham_c<C, +1, true>(Inv{}, v0, t, rowact, row, 1, twl);
            const double w0 = weights ? weights[k] : 1.0;
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] += w0 * (v0[e].x * v0[e].x + v0[e].y * v0[e].y);
            if (!PAIR) {
                wave_lds_sync();
                if (rowact)
#pragma unroll
                    for (int e = 0; e < E; ++e) stash[e] = acc[e];
            }
            if (PAIR && two) {
                wave_lds_sync();
                stockham_c<C, +1, true>(Inv{}, v1, t, rowact, row, 1, twl);
                const double w1 = weights ? weights[k + 1] : 1.0;
#pragma unroll
                for (int e = 0; e < E; ++e) acc[e] += w1 * (v1[e].x * v1[e].x + v1[e].y * v1[e].y);
            }
        }
        __syncthreads();
    }
    if (rowact) {
        double *o = part + (size_t)g * N * N * N3 + (((size_t)z * N + slot) * T + t) * E;
#pragma unroll
        for (int e = 0; e < E; ++e) o[e] = acc[e];
    }
}

// rho[x][y][z] (+)= sum_g part[g] over the groups of one chunk, in group
// order, from the row-thread order of k_plane_density to C order.  One
// work-group per (y, block of kRedZ planes); the block is transposed
// through LDS so that both the partial reads and the rho writes are runs
// of consecutive addresses.
constexpr int kRedZ = 16;
template <int N>
__global__ void __launch_bounds__(256)
k_density_reduce(const double *__restrict__ part, int ngroups, int N3, int accumulate, double *__restrict__ rho)
{
    using C = PlaneCfgP<N, double2>;
    constexpr int T = C::T, E = C::E, RL = ListInfo<typename C::Inv>::last;
    __shared__ double tile[N * (kRedZ + 1)];
    const int y = blockIdx.x, z0 = blockIdx.y * kRedZ;
    const int nz = min(kRedZ, N3 - z0);
    const size_t gstride = (size_t)N * N * N3;
    for (int idx = threadIdx.x; idx < nz * N; idx += 256) {
        const int zz = idx / N, q = idx - zz * N;
        const int t = q / E, e = q - t * E;
        const int x = xlane_rows<N, double2>() ? xl_index<N>(t, e) : t + T * (e / RL) + (e % RL) * (N / RL);
        const double *p = part + ((size_t)(z0 + zz) * N + y) * N + q;
        double s = 0.0;
        for (int gi = 0; gi < ngroups; ++gi) s += p[gi * gstride];
        tile[x * (kRedZ + 1) + zz] = s;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nz * N; idx += 256) {
        const int x = idx / nz, zz = idx - x * nz;
        double *o = rho + ((size_t)x * N + y) * N3 + z0 + zz;
        const double v = tile[x * (kRedZ + 1) + zz];
        *o = accumulate ? *o + v : v;
    }
}

// Potential in the row-thread order of k_plane<N, C2, V>: out[((z N + y) T + t) E + e]
// = V(i1 = x(t, e), i2 = y, i3 = z), x(t, e) = t + T (e / RL) + (e % RL)(N / RL)
// after the Stockham passes, xlane_index(t, e) after the cross-lane rows;
// from vloc in C order [i1][i2][i3].
template <int N, class C2, int V> int plane_x(int t, int e)
{
    using C = PlaneSched<N, C2, V>;
    constexpr int T = C::T, RL = ListInfo<typename C::Inv>::last;
    if constexpr (xlane_pair<N, C2, V>()) return xlane_index(2 * t + e / 12, e % 12);
    else if constexpr (xlane_rows<N, C2>()) return xl_index<N>(t, e);
    else return t + T * (e / RL) + (e % RL) * (N / RL);
}
template <int N, class VT>
void plane_potential(const int32_t *grid, const double *vloc, VT *out)
{
    using C2 = typename std::conditional<std::is_same<VT, float>::value, float2, double2>::type;
    using C = PlaneSched<N, C2, 0>;
    constexpr int T = C::T, E = C::E;
    const int N2 = grid[1], N3 = grid[2];
    for (int z = 0; z < N3; ++z)
        for (int y = 0; y < N2; ++y)
            for (int t = 0; t < T; ++t)
                for (int e = 0; e < E; ++e) {
                    const int x = plane_x<N, C2, 0>(t, e);
                    out[(((size_t)z * N + y) * T + t) * E + e] = (VT)vloc[((size_t)x * N2 + y) * N3 + z];
                }
}
// n1 index of every row position p = t E + e of schedule V
template <int N, class C2> bool row_order(int V, int32_t *x)
{
    auto fill = [&](auto vc) {
        constexpr int VV = decltype(vc)::value;
        using C = PlaneSched<N, C2, VV>;
        for (int t = 0; t < C::T; ++t)
            for (int e = 0; e < C::E; ++e) x[t * C::E + e] = plane_x<N, C2, VV>(t, e);
    };
    if (V < 0 || V >= plane_nsched(N)) return false;
    with_sched<N>(V, fill);
    return true;
}

// Sticks -> sphere, forward transform along n3, then
// out = scale * local + (kin - shift_b) x; dot_part gets sum Re(conj(x) out).
template <int N3, class C2>
__device__ __forceinline__ void stick_fwd_body(int bx, int by, const C2 *__restrict__ sticks, int nst,
                                               const int32_t *__restrict__ st_start,
                                               const int32_t *__restrict__ pt_sz, const C2 *__restrict__ tw,
                                               const C2 *__restrict__ xin, int64_t ld, C2 *__restrict__ out,
                                               const double *__restrict__ kin, const double *__restrict__ shift,
                                               double scale, double *__restrict__ dot_part, int part_stride)
{
    using C = FftCfg<N3>;
    using Fwd = typename C::Fwd;
    using S2 = RealOf<C2>;
    constexpr int NT = stick_threads<N3, C2>();
    constexpr int T = C::T, E = C::E, S = NT / T, LD = N3 + 1;
    __shared__ C2 tile[S * LD];
    __shared__ double red[NT / 64];
    __shared__ C2 twl[N3];  // LDS copy of the twiddle table
    const int tid = threadIdx.x, sl = line_of<T>(tid), t = thread_in_line<T>(tid);
    const int s0 = bx * S, band = by;
    const int s = s0 + sl;
    const bool act = s < nst;
    const C2 *in = sticks + (size_t)band * N3 * nst;
    for (int i = tid; i < N3; i += NT) twl[i] = tw[i];
    __syncthreads();
    C2 v[E];
    C2 *line = tile + sl * LD;
    if constexpr (xlane_rows<N3, C2>()) {
        // cross-lane transform: inputs read in the schedule's register order
        // (zero past the last stick), outputs x[t + T m]
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = act ? in[(size_t)xl_index<N3>(t, e) * nst + s] : cmk<C2>(0.0, 0.0);
        xl_forward<N3>(v, opaque(t), twl);
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (xl_kept<N3>(m)) line[t + T * m] = v[m];
    } else {
        if (act) pass_load<N3, T, E, ListInfo<Fwd>::first>(v, t, [&](int i) { return in[(size_t)i * nst + s]; });
        stockham<N3, -1, true>(Fwd{}, v, t, act, line, 1, twl);
        wave_lds_sync();
        if (act) final_foreach<N3, T, E, ListInfo<Fwd>::last>(v, t, [&](int i, int e) { line[i] = v[e]; });
    }
    __syncthreads();
    const int p0 = st_start[s0], p1 = st_start[min(s0 + S, nst)];
    const double sig = shift ? shift[band] : 0.0;
    const C2 *x = xin + band * ld;
    C2 *o = out + band * ld;
    const S2 sc = (S2)scale;
    double dot = 0.0;
    // loads of kGatherPts points per thread first, as in the sphere scatter;
    // the points are taken, and summed into dot, in the same order as one
    // at a time
    for (int base = p0 + tid; base < p1; base += kGatherPts * NT) {
        int sz[kGatherPts];
        C2 xv[kGatherPts];
        double kv[kGatherPts];
#pragma unroll
        for (int u = 0; u < kGatherPts; ++u) {
            const int idx = base + u * NT, i = idx < p1 ? idx : p0;
            sz[u] = pt_sz[i];
            xv[u] = x[i];
            kv[u] = kin[i];
        }
#pragma unroll
        for (int u = 0; u < kGatherPts; ++u) {
            const int idx = base + u * NT;
            if (idx >= p1) break;
            const C2 loc = tile[((sz[u] >> 8) - s0) * LD + (sz[u] & 255)];
            const S2 k = (S2)(kv[u] - sig);
            C2 r;
            r.x = loc.x * sc + k * xv[u].x;
            r.y = loc.y * sc + k * xv[u].y;
            o[idx] = r;
            dot += (double)xv[u].x * (double)r.x + (double)xv[u].y * (double)r.y;
        }
    }
    if (dot_part) {
        dot = block_sum<NT>(dot, red);
        if (tid == 0) dot_part[(size_t)band * part_stride + bx] = dot;
    }
}
template <int N3, class C2>
__global__ void __launch_bounds__((stick_threads<N3, C2>()))
k_stick_fwd(const C2 *__restrict__ sticks, int nst, const int32_t *__restrict__ st_start,
            const int32_t *__restrict__ pt_sz, const C2 *__restrict__ tw, const C2 *__restrict__ xin, int64_t ld,
            C2 *__restrict__ out, const double *__restrict__ kin, const double *__restrict__ shift, double scale,
            double *__restrict__ dot_part, int part_stride)
{
    stick_fwd_body<N3, C2>(blockIdx.x, blockIdx.y, sticks, nst, st_start, pt_sz, tw, xin, ld, out, kin, shift, scale,
                           dot_part, part_stride);
}
template <int N3, class C2>
__global__ void __launch_bounds__((stick_threads<N3, C2>())) k_stick_fwd_grp(GroupTab t)
{
    int e, bx, by;
    group_block(t, e, bx, by);
    const StickFwdArgs<C2> &a = *static_cast<const StickFwdArgs<C2> *>(t.args[e]);
    stick_fwd_body<N3, C2>(bx, by, a.sticks, a.nst, a.st_start, a.pt_sz, a.tw, a.xin, a.ld, a.out, a.kin, a.shift,
                           a.scale, a.dot_part, a.part_stride);
}


// Precision-specific plan tables.
template <class C2> struct PlanTabs;
template <> struct PlanTabs<double2> {
    static const double2 *tw(const Plan &pl, int d) { return pl.tw[d]; }
    static const double *v(const Plan &pl) { return pl.vplane; }
};
template <> struct PlanTabs<float2> {
    static const float2 *tw(const Plan &pl, int d) { return pl.tw32[d]; }
    static const float *v(const Plan &pl) { return pl.vplane32; }
};
template <class C2> constexpr int prec_index() { return sizeof(C2) == 8 ? 1 : 0; }

// The plane kernel on cb bands of the stick buffer with the plan's line
// schedule and bands per work-group for this precision.
template <int N, class C2>
void launch_plane(const Plan &pl, C2 *sticks, int cb)
{
    const int V = pl.plane_sched[prec_index<C2>()], bpb = pl.plane_bands[prec_index<C2>()];
    const int N3 = pl.grid[2];
    const dim3 grid(N3, (cb + bpb - 1) / bpb);
    auto go = [&](auto vc) {
        constexpr int VV = decltype(vc)::value;
        hipLaunchKernelGGL((k_plane<N, C2, VV>), grid, dim3(plane_threads<N, C2, VV>()), 0, pl.stream, sticks, pl.nst,
                           N3, cb, pl.cols, PlanTabs<C2>::v(pl), pl.nmax[0], PlanTabs<C2>::tw(pl, 0), bpb);
    };
    with_sched<N>(V, go);
}

template <int N, class C2>
hipError_t run_local(const Plan &pl, const Workspace &w, int nb, const C2 *src, int64_t ld, C2 *out,
                     const double *shift, C2 *pbuf, const double *beta, bool first, double *dot_part,
                     int *nparts_out)
{
    // the pruned 96-point transforms leave out the line entries |n| > 23
    if (N == 96 && kXlanePrune && (pl.nmax[0] > 23 || pl.nmax[1] > 23 || pl.nmax[2] > 23))
        return hipErrorInvalidValue;
    constexpr int NT = stick_threads<N, C2>();
    constexpr int S = NT / FftCfg<N>::T;
    const int N3 = pl.grid[2];
    const int ntiles = (pl.nst + S - 1) / S;
    if (nparts_out) *nparts_out = ntiles;
    const double scale = 1.0 / ((double)pl.grid[0] * pl.grid[1] * pl.grid[2]);
    C2 *sticks = reinterpret_cast<C2 *>(w.sticks);
    for (int c0 = 0; c0 < nb; c0 += chunk_bands<C2>()) {
        const int cb = min(chunk_bands<C2>(), nb - c0);
        prof_mark(PARO_K_STICK_INV, pl.stream, true);
        hipLaunchKernelGGL((k_stick_inv<N, C2>), dim3(ntiles, cb), dim3(NT), 0, pl.stream,
                           src + c0 * ld, ld, pbuf ? pbuf + c0 * ld : nullptr, beta ? beta + c0 : nullptr,
                           first ? 1 : 0, sticks, pl.nst, pl.st_start, pl.pt_sz, PlanTabs<C2>::tw(pl, 2));
        prof_mark(PARO_K_STICK_INV, pl.stream, false);
        prof_mark(PARO_K_PLANE, pl.stream, true);
        launch_plane<N, C2>(pl, sticks, cb);
        prof_mark(PARO_K_PLANE, pl.stream, false);
        const C2 *x = pbuf ? pbuf : src;
        prof_mark(PARO_K_STICK_FWD, pl.stream, true);
        hipLaunchKernelGGL((k_stick_fwd<N, C2>), dim3(ntiles, cb), dim3(NT), 0, pl.stream, sticks,
                           pl.nst, pl.st_start, pl.pt_sz, PlanTabs<C2>::tw(pl, 2), x + c0 * ld, ld, out + c0 * ld,
                           pl.kin, shift ? shift + c0 : nullptr, scale,
                           dot_part ? dot_part + (size_t)c0 * kMaxParts : nullptr, kMaxParts);
        prof_mark(PARO_K_STICK_FWD, pl.stream, false);
    }
    return hipGetLastError();
}

// The local part at grids above 96 points: sticks, the plane stage with the
// compressed plane in LDS (k_plane_cc, writing the forward sticks to a
// second stick buffer), the forward sticks.
template <int N, class C2>
hipError_t run_local_big(const Plan &pl, const Workspace &w, int nb, const C2 *src, int64_t ld, C2 *out,
                         const double *shift, C2 *pbuf, const double *beta, bool first, double *dot_part,
                         int *nparts_out)
{
    constexpr int NT = stick_threads<N, C2>();
    constexpr int S = NT / FftCfg<N>::T;
    const int N3 = pl.grid[2];
    const int ntiles = (pl.nst + S - 1) / S;
    if (nparts_out) *nparts_out = ntiles;
    if (pl.ncol > kCcMaxCols) return hipErrorInvalidValue;
    // the pruned lines leave out the entries |n| > 39
    if (kXlanePrune && (pl.nmax[0] > xl_nmax_limit(N) || pl.nmax[1] > xl_nmax_limit(N) ||
                        pl.nmax[2] > xl_nmax_limit(N)))
        return hipErrorInvalidValue;
    const double scale = 1.0 / ((double)pl.grid[0] * pl.grid[1] * pl.grid[2]);
    C2 *sticks = reinterpret_cast<C2 *>(w.sticks);
    C2 *sticks2 = reinterpret_cast<C2 *>(w.sticks2);
    for (int c0 = 0; c0 < nb; c0 += chunk_bands<C2>()) {
        const int cb = min(chunk_bands<C2>(), nb - c0);
        prof_mark(PARO_K_STICK_INV, pl.stream, true);
        hipLaunchKernelGGL((k_stick_inv<N, C2>), dim3(ntiles, cb), dim3(NT), 0, pl.stream, src + c0 * ld, ld,
                           pbuf ? pbuf + c0 * ld : nullptr, beta ? beta + c0 : nullptr, first ? 1 : 0, sticks, pl.nst,
                           pl.st_start, pl.pt_sz, PlanTabs<C2>::tw(pl, 2));
        prof_mark(PARO_K_STICK_INV, pl.stream, false);
        prof_mark(PARO_K_PLANE, pl.stream, true);
        hipLaunchKernelGGL((k_plane_cc<N, C2>), dim3(N3, (cb + kCcBands - 1) / kCcBands), dim3(CcCfg<N, C2>::threads), 0,
                           pl.stream, sticks, sticks2, pl.nst, N3, cb, pl.cols, pl.ncol, pl.nmax[0],
                           PlanTabs<C2>::v(pl), PlanTabs<C2>::tw(pl, 0));
        prof_mark(PARO_K_PLANE, pl.stream, false);
        const C2 *x = pbuf ? pbuf : src;
        prof_mark(PARO_K_STICK_FWD, pl.stream, true);
        hipLaunchKernelGGL((k_stick_fwd<N, C2>), dim3(ntiles, cb), dim3(NT), 0, pl.stream, sticks2, pl.nst,
                           pl.st_start, pl.pt_sz, PlanTabs<C2>::tw(pl, 2), x + c0 * ld, ld, out + c0 * ld, pl.kin,
                           shift ? shift + c0 : nullptr, scale,
                           dot_part ? dot_part + (size_t)c0 * kMaxParts : nullptr, kMaxParts);
        prof_mark(PARO_K_STICK_FWD, pl.stream, false);
    }
    return hipGetLastError();
}

template <int N>
hipError_t run_density(const Plan &pl, double2 *sticks, double *part, int nb, const double2 *psi, int64_t ld,
                       const double *weights, double *rho, bool accumulate)
{
    constexpr int NT = stick_threads<N, double2>();
    constexpr int S = NT / FftCfg<N>::T;
    const int N3 = pl.grid[2];
    const int ntiles = (pl.nst + S - 1) / S;
    for (int c0 = 0; c0 < nb; c0 += kMaxBandsPerChunk) {
        const int cb = min(kMaxBandsPerChunk, nb - c0);
        const int ng = (cb + kDensityBandsPerGroup - 1) / kDensityBandsPerGroup;
        hipLaunchKernelGGL((k_stick_inv<N, double2>), dim3(ntiles, cb), dim3(NT), 0, pl.stream,
                           psi + c0 * ld, ld, nullptr, nullptr, 0, sticks, pl.nst, pl.st_start, pl.pt_sz, pl.tw[2]);
        prof_mark(PARO_K_DENSITY, pl.stream, true);
        hipLaunchKernelGGL((k_plane_density<N>), dim3(N3, ng), dim3(plane_threads<N, double2>()), 0, pl.stream,
                           sticks, pl.nst, N3, cb, kDensityBandsPerGroup, pl.cols, pl.nmax[0],
                           weights ? weights + c0 : nullptr, pl.tw[0], part);
        prof_mark(PARO_K_DENSITY, pl.stream, false);
        hipLaunchKernelGGL((k_density_reduce<N>), dim3(N, (N3 + kRedZ - 1) / kRedZ), dim3(256), 0, pl.stream, part,
                           ng, N3, (accumulate || c0 > 0) ? 1 : 0, rho);
    }
    return hipGetLastError();
}

template <class C2>
hipError_t local_apply(const Plan &pl, const Workspace &w, int nb, const C2 *src, int64_t ld, C2 *out,
                       const double *shift, C2 *pbuf, const double *beta, bool first, double *dot_part,
                       int *nparts_out)
{
    // the kernels are instantiated for cubic grids N1 = N2 = N3
    switch (pl.grid[0]) {
#define PARO_CASE(n) \
    case n: return run_local<n, C2>(pl, w, nb, src, ld, out, shift, pbuf, beta, first, dot_part, nparts_out);
    PARO_CASE(8) PARO_CASE(16) PARO_CASE(24) PARO_CASE(32) PARO_CASE(40) PARO_CASE(48) PARO_CASE(64)
    PARO_CASE(80) PARO_CASE(96)
#undef PARO_CASE
    case 160: return run_local_big<160, C2>(pl, w, nb, src, ld, out, shift, pbuf, beta, first, dot_part, nparts_out);
    default: return hipErrorInvalidValue;
    }
}

template <class C2> hipError_t plane_only(const Plan &pl, const Workspace &w, int nb)
{
    C2 *sticks = reinterpret_cast<C2 *>(w.sticks);
    for (int c0 = 0; c0 < nb; c0 += chunk_bands<C2>()) {
        const int cb = min(chunk_bands<C2>(), nb - c0);
        switch (pl.grid[0]) {
#define PARO_CASE(n) \
    case n: launch_plane<n, C2>(pl, sticks, cb); break;
            PARO_CASE(8) PARO_CASE(16) PARO_CASE(24) PARO_CASE(32) PARO_CASE(40) PARO_CASE(48) PARO_CASE(64)
            PARO_CASE(80) PARO_CASE(96)
#undef PARO_CASE
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

template <class C2> bool row_order_rt(int n, int V, int32_t *x)
{
    switch (n) {
#define PARO_CASE(k) \
    case k: return row_order<k, C2>(V, x);
    PARO_CASE(8) PARO_CASE(16) PARO_CASE(24) PARO_CASE(32) PARO_CASE(40) PARO_CASE(48) PARO_CASE(64)
    PARO_CASE(80) PARO_CASE(96)
#undef PARO_CASE
    default: return false;
    }
}

}  // namespace

int plane_schedules(int n) { return fft_supported(n) && !big_grid(n) ? plane_nsched(n) : 1; }

bool plane_row_map(int n, bool fp32, int from, int to, int32_t *map)
{
    std::vector<int32_t> xf(n), xt(n), pos(n, -1);
    const bool ok = fp32 ? row_order_rt<float2>(n, from, xf.data()) && row_order_rt<float2>(n, to, xt.data())
                         : row_order_rt<double2>(n, from, xf.data()) && row_order_rt<double2>(n, to, xt.data());
    if (!ok) return false;
    for (int p = 0; p < n; ++p) {
        if (xf[p] < 0 || xf[p] >= n || pos[xf[p]] >= 0) return false;
        pos[xf[p]] = p;
    }
    for (int p = 0; p < n; ++p) {
        if (xt[p] < 0 || xt[p] >= n || pos[xt[p]] < 0) return false;
        map[p] = pos[xt[p]];
    }
    return true;
}

hipError_t launch_plane_only(const Plan &pl, const Workspace &w, int nb, bool fp32)
{
    if (big_grid(pl.grid[0])) return hipErrorInvalidValue;
    return fp32 ? plane_only<float2>(pl, w, nb) : plane_only<double2>(pl, w, nb);
}

bool fft_supported(int n)
{
    switch (n) {
    case 8: case 16: case 24: case 32: case 40: case 48: case 64: case 80: case 96: case 160: return true;
    default: return false;
    }
}

bool big_grid(int n) { return n > 96; }

hipError_t launch_density(const Plan &pl, double2 *sticks, double *part, int nb, const double2 *psi, int64_t ld,
                          const double *weights, double *rho, bool accumulate)
{
    switch (pl.grid[0]) {
#define PARO_CASE(n) \
    case n: return run_density<n>(pl, sticks, part, nb, psi, ld, weights, rho, accumulate);
    PARO_CASE(8) PARO_CASE(16) PARO_CASE(24) PARO_CASE(32) PARO_CASE(40) PARO_CASE(48) PARO_CASE(64)
    PARO_CASE(80) PARO_CASE(96)
#undef PARO_CASE
    default: return hipErrorInvalidValue;
    }
}

template <class VT> static void build_plane_potential_t(int n, const int32_t *grid, const double *vloc, VT *out)
{
    switch (n) {
#define PARO_CASE(k) \
    case k: plane_potential<k, VT>(grid, vloc, out); break;
    PARO_CASE(8) PARO_CASE(16) PARO_CASE(24) PARO_CASE(32) PARO_CASE(40) PARO_CASE(48) PARO_CASE(64)
    PARO_CASE(80) PARO_CASE(96) PARO_CASE(160)
#undef PARO_CASE
    default: break;
    }
}

void build_plane_potential(int n, const int32_t *grid, const double *vloc, double *out)
{
    build_plane_potential_t(n, grid, vloc, out);
}

void build_plane_potential(int n, const int32_t *grid, const double *vloc, float *out)
{
    build_plane_potential_t(n, grid, vloc, out);
}

hipError_t launch_local_apply(const Plan &pl, const Workspace &w, int nb, const double2 *src, int64_t ld,
                              double2 *out, const double *shift, double2 *pbuf, const double *beta, bool first,
                              double *dot_part, int *nparts_out)
{
    return local_apply<double2>(pl, w, nb, src, ld, out, shift, pbuf, beta, first, dot_part, nparts_out);
}

hipError_t launch_local_apply(const Plan &pl, const Workspace &w, int nb, const float2 *src, int64_t ld, float2 *out,
                              const double *shift, float2 *pbuf, const double *beta, bool first, double *dot_part,
                              int *nparts_out)
{
    return local_apply<float2>(pl, w, nb, src, ld, out, shift, pbuf, beta, first, dot_part, nparts_out);
}

}  // namespace paro

namespace paro {

// ---------------------------------------------------------------- grouped launches
// The local part of the source solve's (H - sigma) p for many cells: per
// 64-band chunk the arguments run_local gives k_stick_inv, k_plane and
// k_stick_fwd, with src = z, out = q, pbuf = p, beta = the PCG beta.
int describe_local_apply(const Plan &pl, const Workspace &w, int nb, const double *shift, GroupCellDesc &d)
{
    const int N3 = pl.grid[2];
    int ntiles = 0;
    const double scale = 1.0 / ((double)pl.grid[0] * pl.grid[1] * pl.grid[2]);
    const double *beta = w.sc + SC_BETA * nb;
    double *pq_parts = w.dots + (size_t)DOT_PQ * nb * kMaxParts;
    float2 *sticks32 = reinterpret_cast<float2 *>(w.sticks);
    for (int c = 0, c0 = 0; c0 < nb; ++c, c0 += chunk_bands<double2>()) {
        const int cb = std::min(chunk_bands<double2>(), nb - c0);
        const int64_t o = (int64_t)c0 * pl.ldv;
        const double *sh = shift ? shift + c0 : nullptr;
        double *dp = pq_parts + (size_t)c0 * kMaxParts;
        d.f64.sinv[c] = StickInvArgs<double2>{w.z + o, pl.ldv, w.p + o, beta + c0, w.sticks, pl.st_start, pl.pt_sz,
                                              pl.tw[2], pl.nst};
        d.f64.plane[c] = PlaneArgs<double2>{w.sticks, pl.cols, pl.vplane, pl.tw[0], pl.nst, N3, cb, pl.nmax[0],
                                            pl.plane_bands[0]};
        d.f64.sfwd[c] = StickFwdArgs<double2>{w.sticks, pl.st_start, pl.pt_sz, pl.tw[2], w.p + o, pl.ldv, w.q + o,
                                              pl.kin, sh, scale, dp, pl.nst, kMaxParts};
    }
    for (int c = 0, c0 = 0; c0 < nb; ++c, c0 += chunk_bands<float2>()) {
        const int cb = std::min(chunk_bands<float2>(), nb - c0);
        const int64_t o = (int64_t)c0 * pl.ldv;
        const double *sh = shift ? shift + c0 : nullptr;
        double *dp = pq_parts + (size_t)c0 * kMaxParts;
        d.f32.sinv[c] = StickInvArgs<float2>{w.z32 + o, pl.ldv, w.p32 + o, beta + c0, sticks32, pl.st_start,
                                             pl.pt_sz, pl.tw32[2], pl.nst};
        d.f32.plane[c] = PlaneArgs<float2>{sticks32, pl.cols, pl.vplane32, pl.tw32[0], pl.nst, N3, cb, pl.nmax[0],
                                           pl.plane_bands[1]};
        d.f32.sfwd[c] = StickFwdArgs<float2>{sticks32, pl.st_start, pl.pt_sz, pl.tw32[2], w.p32 + o, pl.ldv,
                                             w.q32 + o, pl.kin, sh, scale, dp, pl.nst, kMaxParts};
    }
    switch (pl.grid[0]) {
#define PARO_CASE(n) \
    case n: ntiles = (pl.nst + stick_threads<n, double2>() / FftCfg<n>::T - 1) / (stick_threads<n, double2>() / FftCfg<n>::T); break;
    PARO_CASE(8) PARO_CASE(16) PARO_CASE(24) PARO_CASE(32) PARO_CASE(40) PARO_CASE(48) PARO_CASE(64)
    PARO_CASE(80) PARO_CASE(96)
#undef PARO_CASE
    default: break;
    }
    return ntiles;
}

bool grouped_grid(int n) { return fft_supported(n) && !big_grid(n); }

namespace {

// FIN: the arguments of W = H U at the end of an outer iteration (FP64)
// instead of those of the source solve
template <int N, class C2, bool FIN>
hipError_t grouped_local_n(hipStream_t s, const GroupCell *cells, int n, bool first)
{
    constexpr int NT = stick_threads<N, C2>();
    constexpr int S = NT / FftCfg<N>::T;
    // chunks of this precision's size (FP64 and FP32 passes take different numbers of bands)
    constexpr int CB = chunk_bands<C2>();
    auto nchunk = [](const GroupCell &c) { return (c.nb + CB - 1) / CB; };
    int rounds = 0;
    for (int i = 0; i < n; ++i)
        if (cells[i].pl->grid[0] == N) rounds = std::max(rounds, nchunk(cells[i]));
    for (int i = 0; i < n; ++i)
        if (N == 96 && kXlanePrune && cells[i].pl->grid[0] == N &&
            (cells[i].pl->nmax[0] > 23 || cells[i].pl->nmax[1] > 23 || cells[i].pl->nmax[2] > 23))
            return hipErrorInvalidValue;
    constexpr int pi = prec_index<C2>();
    for (int r = 0; r < rounds; ++r) {
        // the three kernels in turn, every entry of the round in each (the
        // plane kernel once per line schedule the cells use)
        constexpr int nv = plane_nsched(N);
        for (int step = 0; step < nv + 2; ++step) {
            const int k = step == 0 ? 0 : (step <= nv ? 1 : 2), V = k == 1 ? step - 1 : 0;
            GroupBuilder g;
            auto flush = [&]() {
                if (g.t.n == 0) return;
                const dim3 grid((unsigned)g.total);
                if (k == 0)
                    hipLaunchKernelGGL((k_stick_inv_grp<N, C2>), grid, dim3(NT), 0, s, g.t, first ? 1 : 0);
                else if (k == 1) {
                    auto go = [&](auto vc) {
                        constexpr int VV = decltype(vc)::value;
                        hipLaunchKernelGGL((k_plane_grp<N, C2, VV>), grid, dim3(plane_threads<N, C2, VV>()), 0, s,
                                           g.t);
                    };
                    with_sched<N>(V, go);
                } else
                    hipLaunchKernelGGL((k_stick_fwd_grp<N, C2>), grid, dim3(NT), 0, s, g.t);
                g = GroupBuilder();
            };
            for (int i = 0; i < n; ++i) {
                const GroupCell &c = cells[i];
                if (c.pl->grid[0] != N || nchunk(c) <= r) continue;
                if (k == 1 && c.pl->plane_sched[pi] != V) continue;
                const int cb = std::min(CB, c.nb - r * CB);
                const int ntiles = (c.pl->nst + S - 1) / S;
                const void *ai, *ap, *af;
                if constexpr (FIN) {
                    ai = &c.dev->fin.sinv[r];
                    ap = &c.dev->fin.plane[r];
                    af = &c.dev->fin.sfwd[r];
                } else {
                    const GroupSolveArgs<C2> *a = group_solve_args<C2>(c.dev);
                    ai = &a->sinv[r];
                    ap = &a->plane[r];
                    af = &a->sfwd[r];
                }
                if (k == 0) g.add(ai, (int64_t)ntiles * cb, ntiles);
                else if (k == 1) {
                    const int bpb = c.pl->plane_bands[pi];
                    g.add(ap, (int64_t)c.pl->grid[2] * ((cb + bpb - 1) / bpb), c.pl->grid[2]);
                }
                else g.add(af, (int64_t)ntiles * cb, ntiles);
                if (g.full()) flush();
            }
            flush();
        }
    }
    return hipGetLastError();
}

}  // namespace

template <class C2> hipError_t launch_local_apply_grouped(hipStream_t s, const GroupCell *cells, int n, bool first)
{
    hipError_t e = hipSuccess;
#define PARO_CASE(k) \
    if (e == hipSuccess) e = grouped_local_n<k, C2, false>(s, cells, n, first);
    PARO_CASE(8) PARO_CASE(16) PARO_CASE(24) PARO_CASE(32) PARO_CASE(40) PARO_CASE(48) PARO_CASE(64)
    PARO_CASE(80) PARO_CASE(96)
#undef PARO_CASE
    return e;
}
template hipError_t launch_local_apply_grouped<double2>(hipStream_t, const GroupCell *, int, bool);

// W = H U, local part (launch_local_apply(U, W) without PCG prologue, shift or dot products)
void describe_finish_local(const Plan &pl, const Workspace &w, int nb, const double2 *U, double2 *W, int64_t ld,
                           GroupFinishArgs &f)
{
    const int N3 = pl.grid[2];
    const double scale = 1.0 / ((double)pl.grid[0] * pl.grid[1] * pl.grid[2]);
    for (int c = 0, c0 = 0; c0 < nb; ++c, c0 += chunk_bands<double2>()) {
        const int cb = std::min(chunk_bands<double2>(), nb - c0);
        const int64_t o = (int64_t)c0 * ld;
        f.sinv[c] = StickInvArgs<double2>{U + o, ld, nullptr, nullptr, w.sticks, pl.st_start, pl.pt_sz, pl.tw[2],
                                          pl.nst};
        f.plane[c] = PlaneArgs<double2>{w.sticks, pl.cols, pl.vplane, pl.tw[0], pl.nst, N3, cb, pl.nmax[0],
                                        pl.plane_bands[0]};
        f.sfwd[c] = StickFwdArgs<double2>{w.sticks, pl.st_start, pl.pt_sz, pl.tw[2], U + o, ld, W + o, pl.kin,
                                          nullptr, scale, nullptr, pl.nst, kMaxParts};
    }
}

hipError_t launch_finish_local_grouped(hipStream_t s, const GroupCell *cells, int n)
{
    hipError_t e = hipSuccess;
#define PARO_CASE(k) \
    if (e == hipSuccess) e = grouped_local_n<k, double2, true>(s, cells, n, false);
    PARO_CASE(8) PARO_CASE(16) PARO_CASE(24) PARO_CASE(32) PARO_CASE(40) PARO_CASE(48) PARO_CASE(64)
    PARO_CASE(80) PARO_CASE(96)
#undef PARO_CASE
    return e;
}
template hipError_t launch_local_apply_grouped<float2>(hipStream_t, const GroupCell *, int, bool);

}  // namespace paro
