// Complex double GEMMs on the FP64 matrix cores of gfx950, and the device
// construction of the Kleinman-Bylander projector matrix.
//
// Every complex product is four real matrix-core products: 16 x 4 by 4 x 16
// steps of v_mfma_f64_16x16x4f64 (double2 operands) or
// v_mfma_f32_16x16x4f32 (float2 operands).  Lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; it holds D[l / 16 + 4 v][l % 16], v < 4, for the
// FP64 instruction and D[4 (l / 16) + v][l % 16] for the FP32 one.
//
// gemm_hn: C = A^H B with a long contraction (projector coefficients
// P = B^H psi, Gram matrices U^H U and U^H W of Rayleigh-Ritz).  The
// contraction is split over work-groups; partial tiles are summed in a
// fixed order by a second kernel, so results are bitwise reproducible.
// gemm_nn: C (+)= A B with a tall A and a short contraction (the nonlocal
// add q += B (D P) and the Ritz rotations U C, W C).  The matrix-core tile
// is laid out as (column of C) x (row of C) so that a lane group writes 16
// consecutive rows of C: stores are coalesced along the sphere.
#include <algorithm>
#include <cmath>
#include <vector>

#include "fft_device.h"
#include "group.h"
#include "paro_internal.h"
#include "reduce_device.h"

namespace paro {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// c + (-a) b.  The FP64 instruction negates its A operand itself (the
// blgp field of the FP64 matrix instructions holds the neg:[A,B,C] bits);
// the FP32 one has no such modifier.
__device__ __forceinline__ d4 mfma_nega(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 1);
}
__device__ __forceinline__ f4 mfma_nega(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(-a, b, c, 0, 0, 0);
}

// accumulator type and output row of lane group lk, element v
template <class C2> struct Mma;
template <> struct Mma<double2> {
    using Acc = d4;
    static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <> struct Mma<float2> {
    using Acc = f4;
    static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

namespace {

constexpr int kXcds = 8;    // accelerator complex dies; work-group b runs on die b % kXcds

// Work index of work-group b among total: the work-groups of one die get
// consecutive work indices in dispatch order, so tiles that share operands
// (adjacent work indices) run at the same time on the same die and share
// its L2.  A bijection of [0, total).
__device__ __forceinline__ int64_t xcd_work_index(int64_t b, int64_t total)
{
    const int64_t q = total / kXcds, r = total % kXcds;
    const int64_t x = b % kXcds, l = b / kXcds;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + l;
}
// gemm_hn schedule per operand precision: wavefronts the split products
// spread over and k-steps of 4 in flight per wave (register prefetch
// ring).  FP64: one wave per SIMD with splits twice as long, so that the
// ring may take most of the registers (for the 128 x 160 x 34265
// projector product: 2048 slots and 8 steps 122 us; 1024 slots and 8, 12,
// 16 steps 108, 105, 94 us).  FP32: two waves per SIMD, 8 steps (1024
// slots and 16 steps: 106 against 96 us).
template <class C2> struct HnCfg;
template <> struct HnCfg<double2> {
    static constexpr int slots = 1024, depth = 16;
};
template <> struct HnCfg<float2> {
    static constexpr int slots = 2048, depth = 8;
};
// gemm_nn schedule per operand precision: wavefronts the persistent grid
// holds (2048: two per SIMD) and k-steps in flight per wave for its short
// contraction.  For the 34265 x 160 x 128 nonlocal product (FP64) 2048
// slots and 4 steps took 120 us; 8 steps 136 us; 1024 slots with 4, 8, 16
// steps 124, 133, 148 us.  In FP32, 3072 slots for A B and 4096 for A^H B
// took 77 and 102 (+ 12.7 reduce) us against 76 and 92 (+ 8.3) us, and
// rings of 8 (A B) and 16 (A^H B) steps 79 and 105 us.
template <class C2> struct NnCfg;
template <> struct NnCfg<double2> {
    static constexpr int slots = 2048, depth = 4;
};
template <> struct NnCfg<float2> {
    static constexpr int slots = 2048, depth = 4;
};

// partial[s][j][i] = sum over k in split s of conj(A[k][i]) B[k][j]
// (accumulated in the operands' precision, stored in FP64).  Work unit =
// one 32 x 32 block of one split, done by one wavefront; the wavefronts of
// the grid take the units in turn (unit u, u + waves, ...).  Units of one
// split are adjacent, so the blocks that share the split's slices of A and
// B run at the same time on the same die.
template <class C2>
__device__ __forceinline__ void hn_unit(int64_t unit, int lane, int M, int N, int64_t K, int64_t kchunk, int bm,
                                        int bn, const C2 *__restrict__ A, int64_t lda, const C2 *__restrict__ B,
                                        int64_t ldb, double2 *__restrict__ part)
{
    using Acc = typename Mma<C2>::Acc;
    constexpr int kDepthHN = HnCfg<C2>::depth;
    {
        const int split = (int)(unit / (bm * bn)), blk = (int)(unit % (bm * bn));
        const int i0 = (blk % bm) * 32, j0 = (blk / bm) * 32;
        const int64_t kb = (int64_t)split * kchunk;
        const int64_t ke = kb + kchunk < K ? kb + kchunk : K;
        const int l16 = lane & 15, lk = lane >> 4;
        Acc re[2][2], im[2][2];
    #pragma unroll
        for (int a = 0; a < 2; ++a)
    #pragma unroll
            for (int b = 0; b < 2; ++b) {
                re[a][b] = Acc{0, 0, 0, 0};
                im[a][b] = Acc{0, 0, 0, 0};
            }
        // Rows and columns past M and N read the last valid one: lane l16's
        // A operand only reaches row i0 + l16 of the block and its B operand
        // only column j0 + l16, which are not stored.
        const C2 *pa[2] = {A + (int64_t)min(i0 + l16, M - 1) * lda, A + (int64_t)min(i0 + 16 + l16, M - 1) * lda};
        const C2 *pb[2] = {B + (int64_t)min(j0 + l16, N - 1) * ldb, B + (int64_t)min(j0 + 16 + l16, N - 1) * ldb};
        // Register prefetch ring: the operands of k-step s + kDepthHN - 1 are
        // requested before the products of step s, so that their latency
        // overlaps kDepthHN - 1 steps of matrix-core work.  Operand loads are
        // never under a branch, so that the compiler counts the loads in
        // flight instead of waiting for all of them.
        C2 a[kDepthHN][2], b[kDepthHN][2];
        auto step = [&](int slot) {
    #pragma unroll
            for (int u = 0; u < 2; ++u)
    #pragma unroll
                for (int w = 0; w < 2; ++w) {
                    // conj(a) b = (ar br + ai bi) + i (ar bi - ai br)
                    re[u][w] = mfma(a[slot][u].x, b[slot][w].x, re[u][w]);
                    re[u][w] = mfma(a[slot][u].y, b[slot][w].y, re[u][w]);
                    im[u][w] = mfma(a[slot][u].x, b[slot][w].y, im[u][w]);
                    im[u][w] = mfma_nega(a[slot][u].y, b[slot][w].x, im[u][w]);
                }
        };
        constexpr int ring = 4 * kDepthHN;  // k per pass over the ring
        if (ke - kb == kchunk && kchunk % ring == 0) {
            // Full split: every step and every prefetch lies inside the
            // split, so loads take fixed offsets from four pointers that
            // advance once per pass, and nothing is masked.
            const C2 *qa[2] = {pa[0] + kb + lk, pa[1] + kb + lk};
            const C2 *qb[2] = {pb[0] + kb + lk, pb[1] + kb + lk};
            auto load = [&](int slot, int off) {
    #pragma unroll
                for (int u = 0; u < 2; ++u) {
                    a[slot][u] = qa[u][off];
                    b[slot][u] = qb[u][off];
                }
            };
    #pragma unroll
            for (int d = 0; d < kDepthHN - 1; ++d) {
                // slots issued in ring order, so that the loop's waits count
                // the same loads on its first pass as on the later ones
                load(d, 4 * d);
                __builtin_amdgcn_sched_barrier(0);
            }
            for (int64_t t = kchunk / ring; t > 1; --t) {
    #pragma unroll
                for (int d = 0; d < kDepthHN; ++d) {
                    load((d + kDepthHN - 1) % kDepthHN, 4 * (d + kDepthHN - 1));
                    step(d);
                }
    #pragma unroll
                for (int u = 0; u < 2; ++u) {
                    qa[u] += ring;
                    qb[u] += ring;
                }
            }
            // last pass: only the final step remains to be requested
            load(kDepthHN - 1, 4 * (kDepthHN - 1));
    #pragma unroll
            for (int d = 0; d < kDepthHN; ++d) step(d);
        } else if (kb < ke) {
            // Partial split (the last one, or K not a multiple of the ring):
            // steps past the split's end read the last valid k and their A
            // operand is zeroed where it is used.
            auto load = [&](int slot, int64_t k0) {
                const int64_t kk = k0 + lk < K ? k0 + lk : K - 1;
    #pragma unroll
                for (int u = 0; u < 2; ++u) {
                    a[slot][u] = pa[u][kk];
                    b[slot][u] = pb[u][kk];
                }
            };
    #pragma unroll
            for (int d = 0; d < kDepthHN - 1; ++d) {
                load(d, kb + 4 * d);
                __builtin_amdgcn_sched_barrier(0);
            }
            for (int64_t k0 = kb; k0 < ke; k0 += ring) {
    #pragma unroll
                for (int d = 0; d < kDepthHN; ++d) {
                    load((d + kDepthHN - 1) % kDepthHN, k0 + 4 * (d + kDepthHN - 1));
                    const bool kv = k0 + 4 * d + lk < ke;
    #pragma unroll
                    for (int u = 0; u < 2; ++u)
                        if (!kv) a[d][u] = C2{0, 0};
                    step(d);
                }
            }
        }
        double2 *P = part + (size_t)split * M * N;
    #pragma unroll
        for (int u = 0; u < 2; ++u)
    #pragma unroll
            for (int w = 0; w < 2; ++w)
    #pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = i0 + u * 16 + Mma<C2>::row(lk, v);
                    const int j = j0 + w * 16 + l16;
                    if (i < M && j < N) P[(size_t)j * M + i] = make_double2(re[u][w][v], im[u][w][v]);
                }
    }
}
template <class C2>
__global__ void __launch_bounds__(256)
k_gemm_hn_part(int M, int N, int64_t K, int64_t kchunk, int bm, int bn, int64_t units, const C2 *__restrict__ A,
               int64_t lda, const C2 *__restrict__ B, int64_t ldb, double2 *__restrict__ part)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t unit = xcd_work_index(blockIdx.x, gridDim.x) * 4 + wave; unit < units; unit += nw)
        hn_unit<C2>(unit, lane, M, N, K, kchunk, bm, bn, A, lda, B, ldb, part);
}
// the units of every entry, in one range (start[] counts units)
template <class C2> __global__ void __launch_bounds__(256) k_gemm_hn_part_grp(GroupTab t)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t nw = (int64_t)gridDim.x * 4, total = t.start[t.n];
    for (int64_t g = xcd_work_index(blockIdx.x, gridDim.x) * 4 + wave; g < total; g += nw) {
        const int e = group_entry(t, g);
        const GemmHnArgs<C2> &a = *static_cast<const GemmHnArgs<C2> *>(t.args[e]);
        hn_unit<C2>(g - t.start[e], lane, a.M, a.N, a.K, a.kchunk, a.bm, a.bn, a.A, a.lda, a.B, a.ldb, a.part);
    }
}

// C[i][j] = dscale_i * sum_s part[s][j][i]; quad_j = sum_i dscale_i |sum_s part|^2.
// One work-group per column j; 64 rows at a time, the splits dealt to four
// thread groups (group g sums s = g, g + 4, ... in order) and the four
// group sums added in group order: a fixed summation order, so the result
// is bitwise reproducible, with four times the loads in flight of one
// thread per row.
template <class CO>
__device__ __forceinline__ void hn_reduce_body(int j, int M, int N, int nsplit, const double2 *__restrict__ part,
                                               CO *__restrict__ C, int64_t ldc, const double *__restrict__ dscale,
                                               double *__restrict__ quad)
{
    __shared__ double red[4];
    __shared__ double2 grp[4][64];
    const int r = threadIdx.x & 63, g = threadIdx.x >> 6;
    double q = 0.0;
    for (int i0 = 0; i0 < M; i0 += 64) {
        const int i = i0 + r;
        double2 s = make_double2(0.0, 0.0);
        if (i < M) {
#pragma unroll 4
            for (int p = g; p < nsplit; p += 4) {
                const double2 x = part[((size_t)p * N + j) * M + i];
                s.x += x.x;
                s.y += x.y;
            }
        }
        grp[g][r] = s;
        __syncthreads();
        if (g == 0 && i < M) {
            double2 t = grp[0][r];
#pragma unroll
            for (int k = 1; k < 4; ++k) {
                t.x += grp[k][r].x;
                t.y += grp[k][r].y;
            }
            if (dscale) {
                const double d = dscale[i];
                q += d * (t.x * t.x + t.y * t.y);
                t.x *= d;
                t.y *= d;
            }
            C[(int64_t)j * ldc + i] = cmk<CO>(t.x, t.y);
        }
        __syncthreads();
    }
    if (quad) {
        q = block_sum<256>(q, red);
        if (threadIdx.x == 0) quad[j] = q;
    }
}
template <class CO>
__global__ void __launch_bounds__(256)
k_gemm_hn_reduce(int M, int N, int nsplit, const double2 *__restrict__ part, CO *__restrict__ C, int64_t ldc,
                 const double *__restrict__ dscale, double *__restrict__ quad)
{
    hn_reduce_body<CO>(blockIdx.x, M, N, nsplit, part, C, ldc, dscale, quad);
}
template <class CO> __global__ void __launch_bounds__(256) k_gemm_hn_reduce_grp(GroupTab t)
{
    int e, bx, by;
    group_block(t, e, bx, by);
    const GemmHnRedArgs<CO> &a = *static_cast<const GemmHnRedArgs<CO> *>(t.args[e]);
    hn_reduce_body<CO>(bx, a.M, a.N, a.nsplit, a.part, a.C, a.ldc, a.dscale, a.quad);
}

// C[g][n] (+)= sum_k A[g][k] B[k][n]; matrix-core rows = n, columns = g.
template <class C2>
__device__ __forceinline__ void nn_unit(int64_t unit, int lane, int64_t M, int N, int K, int bn,
                                        const C2 *__restrict__ A, int64_t lda, const C2 *__restrict__ B, int64_t ldb,
                                        C2 *__restrict__ C, int64_t ldc, int accumulate)
{
    using Acc = typename Mma<C2>::Acc;
    constexpr int kDepthNN = NnCfg<C2>::depth;
    {
        const int64_t g0 = (unit / bn) * 32;
        const int n0 = (int)(unit % bn) * 32;
        const int l16 = lane & 15, lk = lane >> 4;
        Acc re[2][2], im[2][2];
    #pragma unroll
        for (int a = 0; a < 2; ++a)
    #pragma unroll
            for (int b = 0; b < 2; ++b) {
                re[a][b] = Acc{0, 0, 0, 0};
                im[a][b] = Acc{0, 0, 0, 0};
            }
        // Lane l16's B operand only reaches row n0 + l16 of C and its A
        // operand only column g0 + l16, so past N and M they read the last
        // valid one (those rows and columns are not stored).
        const C2 *px[2] = {B + (int64_t)min(n0 + l16, N - 1) * ldb, B + (int64_t)min(n0 + 16 + l16, N - 1) * ldb};
        const C2 *py[2] = {A + (g0 + l16 < M ? g0 + l16 : M - 1), A + (g0 + 16 + l16 < M ? g0 + 16 + l16 : M - 1)};
        // Accumulation: the old values of the whole block (clamped into C,
        // as the operand loads) are requested before the last pass of the
        // contraction, so that their latency overlaps its k-steps.
        C2 old[2][2][4];
        auto load_old = [&]() {
            if (!accumulate) return;
    #pragma unroll
            for (int u = 0; u < 2; ++u)
    #pragma unroll
                for (int w = 0; w < 2; ++w)
    #pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int n = min(n0 + u * 16 + Mma<C2>::row(lk, v), N - 1);
                        const int64_t g = g0 + w * 16 + l16 < M ? g0 + w * 16 + l16 : M - 1;
                        old[u][w][v] = C[(int64_t)n * ldc + g];
                    }
        };
        // register prefetch ring, as in k_gemm_hn_part
        C2 x[kDepthNN][2], y[kDepthNN][2];
        auto step = [&](int slot) {
    #pragma unroll
            for (int u = 0; u < 2; ++u)
    #pragma unroll
                for (int w = 0; w < 2; ++w) {
                    // (x y): re = xr yr - xi yi, im = xr yi + xi yr
                    re[u][w] = mfma(x[slot][u].x, y[slot][w].x, re[u][w]);
                    re[u][w] = mfma_nega(x[slot][u].y, y[slot][w].y, re[u][w]);
                    im[u][w] = mfma(x[slot][u].x, y[slot][w].y, im[u][w]);
                    im[u][w] = mfma(x[slot][u].y, y[slot][w].x, im[u][w]);
                }
        };
        constexpr int ring = 4 * kDepthNN;
        if (K % ring == 0) {
            // every step and prefetch inside [0, K): fixed offsets from
            // pointers that advance once per pass, nothing masked
            const C2 *qx[2] = {px[0] + lk, px[1] + lk};
            const C2 *qy[2] = {py[0] + (int64_t)lk * lda, py[1] + (int64_t)lk * lda};
            const int64_t kstep = 4 * lda;
            auto load = [&](int slot, int d) {
    #pragma unroll
                for (int u = 0; u < 2; ++u) {
                    x[slot][u] = qx[u][4 * d];
                    y[slot][u] = qy[u][d * kstep];
                }
            };
    #pragma unroll
            for (int d = 0; d < kDepthNN - 1; ++d) {
                load(d, d);  // in ring order, as in k_gemm_hn_part
                __builtin_amdgcn_sched_barrier(0);
            }
            for (int t = K / ring; t > 1; --t) {
    #pragma unroll
                for (int d = 0; d < kDepthNN; ++d) {
                    load((d + kDepthNN - 1) % kDepthNN, d + kDepthNN - 1);
                    step(d);
                }
    #pragma unroll
                for (int u = 0; u < 2; ++u) {
                    qx[u] += ring;
                    qy[u] += kDepthNN * kstep;
                }
            }
            load(kDepthNN - 1, kDepthNN - 1);
            load_old();
    #pragma unroll
            for (int d = 0; d < kDepthNN; ++d) step(d);
        } else if (K > 0) {
            // steps past K read k = K - 1 and their B operand is zeroed
            auto load = [&](int slot, int k0) {
                const int kk = k0 + lk < K ? k0 + lk : K - 1;
    #pragma unroll
                for (int u = 0; u < 2; ++u) {
                    x[slot][u] = px[u][kk];
                    y[slot][u] = py[u][(int64_t)kk * lda];
                }
            };
    #pragma unroll
            for (int d = 0; d < kDepthNN - 1; ++d) {
                load(d, 4 * d);
                __builtin_amdgcn_sched_barrier(0);
            }
            for (int k0 = 0; k0 < K; k0 += ring) {
    #pragma unroll
                for (int d = 0; d < kDepthNN; ++d) {
                    load((d + kDepthNN - 1) % kDepthNN, k0 + 4 * (d + kDepthNN - 1));
                    const bool kv = k0 + 4 * d + lk < K;
    #pragma unroll
                    for (int u = 0; u < 2; ++u)
                        if (!kv) x[d][u] = C2{0, 0};
                    step(d);
                }
            }
            load_old();
        } else {
            load_old();
        }
    #pragma unroll
        for (int u = 0; u < 2; ++u) {
    #pragma unroll
            for (int w = 0; w < 2; ++w)
    #pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int n = n0 + u * 16 + Mma<C2>::row(lk, v);
                    const int64_t g = g0 + w * 16 + l16;
                    C2 r;
                    r.x = re[u][w][v];
                    r.y = im[u][w][v];
                    if (accumulate) {
                        r.x += old[u][w][v].x;
                        r.y += old[u][w][v].y;
                    }
                    if (n < N && g < M) C[(int64_t)n * ldc + g] = r;
                }
        }
    }
}
template <class C2>
__global__ void __launch_bounds__(256, 2)
k_gemm_nn(int64_t M, int N, int K, int bn, int64_t units, const C2 *__restrict__ A, int64_t lda,
          const C2 *__restrict__ B, int64_t ldb, C2 *__restrict__ C, int64_t ldc, int accumulate)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // work unit = one 32 x 32 block of C, done by one wavefront; the bn
    // column blocks of one row block (which share its rows of A) are
    // adjacent units
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t unit = xcd_work_index(blockIdx.x, gridDim.x) * 4 + wave; unit < units; unit += nw)
        nn_unit<C2>(unit, lane, M, N, K, bn, A, lda, B, ldb, C, ldc, accumulate);
}
template <class C2> __global__ void __launch_bounds__(256, 2) k_gemm_nn_grp(GroupTab t)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t nw = (int64_t)gridDim.x * 4, total = t.start[t.n];
    for (int64_t g = xcd_work_index(blockIdx.x, gridDim.x) * 4 + wave; g < total; g += nw) {
        const int e = group_entry(t, g);
        const GemmNnArgs<C2> &a = *static_cast<const GemmNnArgs<C2> *>(t.args[e]);
        nn_unit<C2>(g - t.start[e], lane, a.M, a.N, a.K, a.bn, a.A, a.lda, a.B, a.ldb, a.C, a.ldc, a.accumulate);
    }
}

// One work-group per projector: beta_p(G) for every sphere point, then the
// normalisation sum_G |beta_p(G)|^2 = 1 (two passes over the sphere).
__global__ void __launch_bounds__(256)
k_build_projectors(int64_t ng, const int32_t *__restrict__ miller, double b00, double b01, double b02,
                   double b10, double b11, double b12, double b20, double b21, double b22,
                   const double *__restrict__ centers, const int32_t *__restrict__ lm,
                   const double *__restrict__ widths, double2 *__restrict__ beta, int64_t ldb)
{
    __shared__ double red[4];
    const int p = blockIdx.x;
    const double R0 = centers[3 * p], R1 = centers[3 * p + 1], R2 = centers[3 * p + 2];
    const int l = lm[2 * p], m = lm[2 * p + 1];
    const double w = widths[p];
    double2 *out = beta + (int64_t)p * ldb;
    double nrm = 0.0;
    for (int64_t g = threadIdx.x; g < ng; g += 256) {
        const double n1 = miller[3 * g], n2 = miller[3 * g + 1], n3 = miller[3 * g + 2];
        const double G0 = n1 * b00 + n2 * b10 + n3 * b20;
        const double G1 = n1 * b01 + n2 * b11 + n3 * b21;
        const double G2 = n1 * b02 + n2 * b12 + n3 * b22;
        const double g2 = G0 * G0 + G1 * G1 + G2 * G2;
        const double gr = G0 * R0 + G1 * R1 + G2 * R2;
        const double env = exp(-0.5 * w * w * g2);
        double sn, cs;
        sincos(gr, &sn, &cs);
        double2 val = make_double2(env * cs, -env * sn);  // exp(-0.5 w^2 G^2) exp(-i G.R)
        if (l == 1) {
            const double ga = m == 0 ? G0 : (m == 1 ? G1 : G2);
            // times (-i w G_a)
            val = make_double2(w * ga * val.y, -w * ga * val.x);
        }
        out[g] = val;
        nrm += val.x * val.x + val.y * val.y;
    }
    nrm = block_sum<256>(nrm, red);
    const double sc = nrm > 0 ? 1.0 / sqrt(nrm) : 0.0;
    for (int64_t g = threadIdx.x; g < ng; g += 256) {
        double2 v = out[g];
        out[g] = make_double2(v.x * sc, v.y * sc);
    }
    for (int64_t g = ng + threadIdx.x; g < ldb; g += 256) out[g] = make_double2(0.0, 0.0);
}

__global__ void __launch_bounds__(256) k_to_single(int64_t n, const double2 *__restrict__ src, float2 *__restrict__ dst)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double2 v = src[i];
        dst[i] = make_float2((float)v.x, (float)v.y);
    }
}

// The split of A^H B over K: about one unit per wavefront slot of the
// chip, each split at least one prefetch ring of k long, within the
// partial buffer, and a whole number of ring passes long (all but the last
// then take the kernel's unmasked path).  False if the buffer is too small.
template <class C2>
bool hn_split(int M, int N, int64_t K, size_t part_elems, int64_t *nsplit_out, int64_t *kchunk_out,
              int64_t *units_out)
{
    const int bm = (M + 31) / 32, bn = (N + 31) / 32;
    constexpr int kDepthHN = HnCfg<C2>::depth, kWaveSlotsHN = HnCfg<C2>::slots;
    int64_t nsplit = kWaveSlotsHN / ((int64_t)bm * bn);
    const int64_t kmax = (K + 4 * kDepthHN - 1) / (4 * kDepthHN);
    if (nsplit > kmax) nsplit = kmax;
    if (nsplit < 1) nsplit = 1;
    const int64_t cap = (int64_t)(part_elems / ((size_t)M * N));
    if (nsplit > cap) nsplit = cap;
    if (nsplit < 1) return false;
    const int64_t ring = 4 * kDepthHN;
    int64_t kchunk = (K + nsplit - 1) / nsplit;
    kchunk = (kchunk + ring - 1) / ring * ring;
    nsplit = (K + kchunk - 1) / kchunk;
    if (nsplit < 1) nsplit = 1;
    *nsplit_out = nsplit;
    *kchunk_out = kchunk;
    *units_out = (int64_t)bm * bn * nsplit;
    return true;
}

template <class C2>
hipError_t gemm_hn_t(hipStream_t s, int M, int N, int64_t K, const C2 *A, int64_t lda, const C2 *B, int64_t ldb,
                     C2 *C, int64_t ldc, double2 *part, size_t part_elems, const double *dscale, double *quad)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    const int bm = (M + 31) / 32, bn = (N + 31) / 32;
    constexpr int kWaveSlotsHN = HnCfg<C2>::slots;
    int64_t nsplit, kchunk, units;
    if (!hn_split<C2>(M, N, K, part_elems, &nsplit, &kchunk, &units)) return hipErrorInvalidValue;
    const unsigned wgs = (unsigned)std::min<int64_t>((units + 3) / 4, kWaveSlotsHN / 4);
    prof_mark(PARO_K_GEMM_HN, s, true);
    hipLaunchKernelGGL((k_gemm_hn_part<C2>), dim3(wgs), dim3(256), 0, s, M, N, K, kchunk, bm, bn, units, A, lda, B,
                       ldb, part);
    prof_mark(PARO_K_GEMM_HN, s, false);
    hipLaunchKernelGGL((k_gemm_hn_reduce<C2>), dim3(N), dim3(256), 0, s, M, N, (int)nsplit, part, C, ldc, dscale,
                       quad);
    return hipGetLastError();
}

template <class C2>
hipError_t gemm_nn_t(hipStream_t s, int64_t M, int N, int K, const C2 *A, int64_t lda, const C2 *B, int64_t ldb,
                     C2 *C, int64_t ldc, bool accumulate)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    const int bn = (N + 31) / 32;
    const int64_t units = (M + 31) / 32 * bn;
    dim3 grid((unsigned)std::min<int64_t>((units + 3) / 4, NnCfg<C2>::slots / 4));
    prof_mark(PARO_K_GEMM_NN, s, true);
    hipLaunchKernelGGL((k_gemm_nn<C2>), grid, dim3(256), 0, s, M, N, K, bn, units, A, lda, B, ldb, C, ldc,
                       accumulate ? 1 : 0);
    prof_mark(PARO_K_GEMM_NN, s, false);
    return hipGetLastError();
}

}  // namespace

hipError_t gemm_hn(hipStream_t s, int M, int N, int64_t K, const double2 *A, int64_t lda, const double2 *B,
                   int64_t ldb, double2 *C, int64_t ldc, double2 *part, size_t part_elems, const double *dscale,
                   double *quad)
{
    return gemm_hn_t(s, M, N, K, A, lda, B, ldb, C, ldc, part, part_elems, dscale, quad);
}

hipError_t gemm_hn(hipStream_t s, int M, int N, int64_t K, const float2 *A, int64_t lda, const float2 *B,
                   int64_t ldb, float2 *C, int64_t ldc, double2 *part, size_t part_elems, const double *dscale,
                   double *quad)
{
    return gemm_hn_t(s, M, N, K, A, lda, B, ldb, C, ldc, part, part_elems, dscale, quad);
}

hipError_t gemm_nn(hipStream_t s, int64_t M, int N, int K, const double2 *A, int64_t lda, const double2 *B,
                   int64_t ldb, double2 *C, int64_t ldc, bool accumulate)
{
    return gemm_nn_t(s, M, N, K, A, lda, B, ldb, C, ldc, accumulate);
}

hipError_t gemm_nn(hipStream_t s, int64_t M, int N, int K, const float2 *A, int64_t lda, const float2 *B,
                   int64_t ldb, float2 *C, int64_t ldc, bool accumulate)
{
    return gemm_nn_t(s, M, N, K, A, lda, B, ldb, C, ldc, accumulate);
}

hipError_t launch_to_single(hipStream_t s, int64_t n, const double2 *src, float2 *dst)
{
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_to_single, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256), 0, s, n, src, dst);
    return hipGetLastError();
}

namespace {

// out[(a n_proj + p) ldv + g] = G_a(g) beta_p(g), G = n1 b1 + n2 b2 + n3 b3.
__global__ void __launch_bounds__(256)
k_gscale_projectors(int64_t ng, int64_t ldv, int np, const int32_t *__restrict__ miller, double b00, double b01,
                    double b02, double b10, double b11, double b12, double b20, double b21, double b22,
                    const double2 *__restrict__ beta, double2 *__restrict__ out)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int p = blockIdx.y;
    if (g >= ng) return;
    const double n1 = miller[3 * g], n2 = miller[3 * g + 1], n3 = miller[3 * g + 2];
    const double G[3] = {n1 * b00 + n2 * b10 + n3 * b20, n1 * b01 + n2 * b11 + n3 * b21,
                         n1 * b02 + n2 * b12 + n3 * b22};
    const double2 v = beta[(int64_t)p * ldv + g];
#pragma unroll
    for (int a = 0; a < 3; ++a) out[((int64_t)a * np + p) * ldv + g] = make_double2(G[a] * v.x, G[a] * v.y);
}

// One work-group per projector; bands summed by thread in a fixed stride
// order, then a fixed-order block reduction.  S^a = (G_a beta)^H psi, so
// Q^a = i S^a and 2 Re(conj(P) Q^a) = -2 Im(conj(P) S^a).
__global__ void __launch_bounds__(256)
k_projector_gradient(int np, int nb, const double2 *__restrict__ P, const double2 *__restrict__ S,
                     const double *__restrict__ weights, const double *__restrict__ dkb, double *__restrict__ dd,
                     double *__restrict__ dR)
{
    __shared__ double red[4];
    const int p = blockIdx.x;
    double sd = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) {
        const double w = weights ? weights[b] : 1.0;
        const double2 pv = P[(int64_t)b * np + p];
        sd += w * (pv.x * pv.x + pv.y * pv.y);
        const double2 q0 = S[(int64_t)b * 3 * np + p];
        const double2 q1 = S[(int64_t)b * 3 * np + np + p];
        const double2 q2 = S[(int64_t)b * 3 * np + 2 * np + p];
        // Im(conj(P) S) = P.x S.y - P.y S.x
        s0 += w * (pv.x * q0.y - pv.y * q0.x);
        s1 += w * (pv.x * q1.y - pv.y * q1.x);
        s2 += w * (pv.x * q2.y - pv.y * q2.x);
    }
    sd = block_sum<256>(sd, red);
    s0 = block_sum<256>(s0, red);
    s1 = block_sum<256>(s1, red);
    s2 = block_sum<256>(s2, red);
    if (threadIdx.x == 0) {
        const double f = -2.0 * dkb[p];
        dd[p] = sd;
        dR[3 * p] = f * s0;
        dR[3 * p + 1] = f * s1;
        dR[3 * p + 2] = f * s2;
    }
}

}  // namespace

hipError_t launch_projector_gradient(const Plan &pl, const ProjGradWs &w, int nb, const double2 *psi, int64_t ld,
                                     const double *weights, double *dd, double *dR)
{
    const int np = pl.nproj;
    if (np == 0) return hipSuccess;
    const double *b = pl.bvec;
    hipLaunchKernelGGL(k_gscale_projectors, dim3((unsigned)((pl.ng + 255) / 256), np), dim3(256), 0, pl.stream, pl.ng,
                       pl.ldv, np, pl.miller, b[0], b[1], b[2], b[3], b[4], b[5], b[6], b[7], b[8], pl.beta, w.gbeta);
    hipError_t e = gemm_hn(pl.stream, np, nb, pl.ng, pl.beta, pl.ldv, psi, ld, w.P, np, w.part, w.part_elems, nullptr,
                           nullptr);
    if (e != hipSuccess) return e;
    e = gemm_hn(pl.stream, 3 * np, nb, pl.ng, w.gbeta, pl.ldv, psi, ld, w.S, 3 * np, w.part, w.part_elems, nullptr,
                nullptr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_projector_gradient, dim3(np), dim3(256), 0, pl.stream, np, nb, w.P, w.S, weights, pl.dkb, dd,
                       dR);
    return hipGetLastError();
}

hipError_t launch_build_projectors(const Plan &pl, const int32_t *miller_dev, const double *centers,
                                   const int32_t *lm, const double *widths)
{
    if (pl.nproj == 0) return hipSuccess;
    const double *b = pl.bvec;
    hipLaunchKernelGGL(k_build_projectors, dim3(pl.nproj), dim3(256), 0, pl.stream, pl.ng, miller_dev, b[0], b[1],
                       b[2], b[3], b[4], b[5], b[6], b[7], b[8], centers, lm, widths, pl.beta, pl.ldv);
    return hipGetLastError();
}

}  // namespace paro

namespace paro {

// ---------------------------------------------------------------- grouped launches
// The nonlocal part of the source solve's (H - sigma) p for many cells: the
// arguments gemm_hn (P = B^H p, times the KB energies, p^H V_NL p into the
// PCG scalars) and gemm_nn (q += B P) give their kernels.
template <class C2>
static void describe_nonlocal_t(const Plan &pl, const Workspace &w, int nb, const C2 *beta, const C2 *p, C2 *q,
                                GroupSolveArgs<C2> &d)
{
    const int M = pl.nproj, N = nb;
    int64_t nsplit = 0, kchunk = 0, units = 0;
    if (M > 0) hn_split<C2>(M, N, pl.ng, w.part_elems, &nsplit, &kchunk, &units);
    C2 *P = reinterpret_cast<C2 *>(w.P);
    d.hn = GemmHnArgs<C2>{beta, pl.ldv, p, pl.ldv, w.part, pl.ng, kchunk, units, M, N, (M + 31) / 32, (N + 31) / 32};
    d.hred = GemmHnRedArgs<C2>{w.part, P, M, pl.dkb, w.sc + SC_NLQ * nb, M, N, (int)nsplit};
    const int bn = (N + 31) / 32;
    d.nn = GemmNnArgs<C2>{beta, pl.ldv, P, M, q, pl.ldv, pl.ng, (pl.ng + 31) / 32 * bn, N, M, bn, 1};
}

void describe_nonlocal(const Plan &pl, const Workspace &w, int nb, GroupCellDesc &d)
{
    describe_nonlocal_t<double2>(pl, w, nb, pl.beta, w.p, w.q, d.f64);
    describe_nonlocal_t<float2>(pl, w, nb, pl.beta32, w.p32, w.q32, d.f32);
}

template <class C2> hipError_t launch_hn_grouped(hipStream_t s, const HnRef<C2> *v, int n)
{
    for (int i0 = 0; i0 < n;) {
        GroupBuilder hn, red;
        int i = i0;
        for (; i < n && !hn.full(); ++i) {
            hn.add(v[i].dev, v[i].host->units, 1);
            red.add(v[i].dred, v[i].host->N, v[i].host->N);
        }
        i0 = i;
        const unsigned w = (unsigned)std::min<int64_t>((hn.total + 3) / 4, HnCfg<C2>::slots / 4);
        hipLaunchKernelGGL((k_gemm_hn_part_grp<C2>), dim3(w), dim3(256), 0, s, hn.t);
        hipLaunchKernelGGL((k_gemm_hn_reduce_grp<C2>), dim3((unsigned)red.total), dim3(256), 0, s, red.t);
    }
    return hipGetLastError();
}

template <class C2> hipError_t launch_nn_grouped(hipStream_t s, const NnRef<C2> *v, int n)
{
    for (int i0 = 0; i0 < n;) {
        GroupBuilder nn;
        int i = i0;
        for (; i < n && !nn.full(); ++i) nn.add(v[i].dev, v[i].host->units, 1);
        i0 = i;
        const unsigned w = (unsigned)std::min<int64_t>((nn.total + 3) / 4, NnCfg<C2>::slots / 4);
        hipLaunchKernelGGL((k_gemm_nn_grp<C2>), dim3(w), dim3(256), 0, s, nn.t);
    }
    return hipGetLastError();
}

template <class C2> hipError_t launch_nonlocal_grouped(hipStream_t s, const GroupCell *cells, int n)
{
    // cells with projectors
    std::vector<HnRef<C2>> hv;
    std::vector<NnRef<C2>> nv;
    for (int i = 0; i < n; ++i) {
        const GroupCell &c = cells[i];
        if (c.pl->nproj == 0) continue;
        const GroupSolveArgs<C2> *a = group_solve_args<C2>(c.dev), *h = group_solve_args<C2>(c.host);
        hv.push_back(HnRef<C2>{&a->hn, &h->hn, &a->hred});
        nv.push_back(NnRef<C2>{&a->nn, &h->nn});
    }
    hipError_t e = launch_hn_grouped<C2>(s, hv.data(), (int)hv.size());
    if (e == hipSuccess) e = launch_nn_grouped<C2>(s, nv.data(), (int)nv.size());
    return e;
}

// The products of W = H U (nonlocal part) and of Rayleigh-Ritz for the
// grouped finish of an outer iteration: as apply_full's gemm_hn / gemm_nn
// on U and rayleigh_ritz's Gram and rotation products.
void describe_finish_products(const Plan &pl, const Workspace &w, int m, int nkeep, const double2 *U,
                              const double2 *W, int64_t ld, double2 *psi, double2 *hpsi, int64_t ldo,
                              GroupFinishArgs &f)
{
    const int np = pl.nproj, bm = (m + 31) / 32;
    int64_t nsplit = 0, kchunk = 0, units = 0;
    if (np > 0) hn_split<double2>(np, m, pl.ng, w.part_elems, &nsplit, &kchunk, &units);
    f.nl_hn = GemmHnArgs<double2>{pl.beta, pl.ldv, U, ld, w.part, pl.ng, kchunk, units, np, m, (np + 31) / 32, bm};
    f.nl_red = GemmHnRedArgs<double2>{w.part, w.P, np, pl.dkb, nullptr, np, m, (int)nsplit};
    f.nl_nn = GemmNnArgs<double2>{pl.beta, pl.ldv, w.P, np, const_cast<double2 *>(W), ld, pl.ng,
                                  (pl.ng + 31) / 32 * bm, m, np, bm, 1};
    hn_split<double2>(m, m, pl.ng, w.part_elems, &nsplit, &kchunk, &units);
    f.s_hn = GemmHnArgs<double2>{U, ld, U, ld, w.part, pl.ng, kchunk, units, m, m, bm, bm};
    f.h_hn = GemmHnArgs<double2>{U, ld, W, ld, w.part, pl.ng, kchunk, units, m, m, bm, bm};
    f.s_red = GemmHnRedArgs<double2>{w.part, w.gram, m, nullptr, nullptr, m, m, (int)nsplit};
    f.h_red = GemmHnRedArgs<double2>{w.part, w.gram + (size_t)m * m, m, nullptr, nullptr, m, m, (int)nsplit};
    const int bk = (nkeep + 31) / 32;
    f.rot_psi = GemmNnArgs<double2>{U, ld, w.dense[4], m, psi, ldo, pl.ng, (pl.ng + 31) / 32 * bk, nkeep, m, bk, 0};
    f.rot_hpsi = GemmNnArgs<double2>{W, ld, w.dense[4], m, hpsi, ldo, pl.ng, (pl.ng + 31) / 32 * bk, nkeep, m, bk, 0};
}

template hipError_t launch_nonlocal_grouped<double2>(hipStream_t, const GroupCell *, int);
template hipError_t launch_nonlocal_grouped<float2>(hipStream_t, const GroupCell *, int);
template hipError_t launch_hn_grouped<double2>(hipStream_t, const HnRef<double2> *, int);
template hipError_t launch_nn_grouped<double2>(hipStream_t, const NnRef<double2> *, int);

}  // namespace paro
