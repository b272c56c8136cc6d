// Projector products of the mixed-precision apply on the BF16 matrix cores
// of gfx950, with each FP32 operand split into two BF16 parts (bf16x3).
//
// A real x is held as hi + lo with hi = bf16(x) and lo = bf16(x - hi), so
// |x - hi - lo| <= 2^-16 |x|.  A product x y is taken as
// hi_x hi_y + hi_x lo_y + lo_x hi_y (the lo lo term, at most 2^-16 |x y|,
// is dropped); the three products run on v_mfma_f32_16x16x32_bf16 with
// FP32 accumulation.  Each product is within about 3 x 2^-16 of x y: the
// nonlocal part of H x carries a relative error of about 5e-5, against
// 6e-8 for FP32 operands, at a third of the matrix-core cycles.
//
// Complex operands are stored as packed BF16 pairs (real part in the low
// half of a 32-bit word), so a contraction over K complex values is a real
// contraction over 2K interleaved values:
//   Re(conj(a) b) = a_r b_r + a_i b_i,   Im(conj(a) b) = rot(a) . b,
//   Re(a y) = a . (y_r, -y_i),           Im(a y) = a . rot(y_r, -y_i),
// with rot(u, v) = (-v, u) on each pair (a word rotate and a sign flip).
//
// Lane l of a 16 x 16 x 32 product supplies row l % 16 of A and column
// l % 16 of B over the 8 interleaved values (4 complex) at k-group l / 16;
// it holds D[4 (l / 16) + v][l % 16], v < 4.  The instruction pairs A's and
// B's values by position, and both operands are loaded with the same
// k-group per lane, so the contraction covers every k once.
//
// Contractions are padded with zeros to whole prefetch-ring passes: the
// kernels run no masked steps.
#include <algorithm>
#include <cstdint>

#include "paro_internal.h"
#include "reduce_device.h"

namespace paro {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

constexpr int kXcdsB = 8;

__device__ __forceinline__ int64_t xcd_index(int64_t b, int64_t total)
{
    const int64_t q = total / kXcdsB, r = total % kXcdsB;
    const int64_t x = b % kXcdsB, l = b / kXcdsB;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + l;
}

__device__ __forceinline__ f4 mma(u4 a, u4 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0,
                                                   0);
}
// (re, im) -> (-im, re) on four packed pairs
__device__ __forceinline__ u4 rot(u4 v)
{
    u4 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = __builtin_amdgcn_alignbit(v[i], v[i], 16) ^ 0x8000u;
    return r;
}

__device__ __forceinline__ uint32_t bf16_bits(float x)
{
    return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)x);
}
__device__ __forceinline__ float bf16_value(float x) { return (float)(__bf16)x; }
// hi and lo words of the pair (a, b)
__device__ __forceinline__ void split_pair(float a, float b, uint32_t &hi, uint32_t &lo)
{
    const float ha = bf16_value(a), hb = bf16_value(b);
    hi = bf16_bits(ha) | (bf16_bits(hb) << 16);
    lo = bf16_bits(a - ha) | (bf16_bits(b - hb) << 16);
}

// Plan tables: the FP64 projectors beta (nproj x ldv, projector-major) as
// hi / lo pairs in the same layout (row length ldk, zero past ng) and
// transposed, [g][p] (row length ldp, zero past nproj).
__global__ void __launch_bounds__(256)
k_split_beta(int64_t ng, int nproj, const double2 *__restrict__ beta, int64_t ldv, int64_t ldk, int ldp,
             uint32_t *__restrict__ bs_hi, uint32_t *__restrict__ bs_lo, uint32_t *__restrict__ bt_hi,
             uint32_t *__restrict__ bt_lo)
{
    const int p = blockIdx.y;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < ldk; g += (int64_t)gridDim.x * 256) {
        uint32_t hi = 0, lo = 0;
        if (p < nproj && g < ng) {
            const double2 v = beta[(size_t)p * ldv + g];
            split_pair((float)v.x, (float)v.y, hi, lo);
        }
        if (p < nproj) {
            bs_hi[(size_t)p * ldk + g] = hi;
            bs_lo[(size_t)p * ldk + g] = lo;
        }
        if (g < ng) {
            bt_hi[(size_t)g * ldp + p] = hi;
            bt_lo[(size_t)g * ldp + p] = lo;
        }
    }
}

// x (nb x ld complex FP32) -> hi / lo pairs (nb x ldk, zero past ng)
__global__ void __launch_bounds__(256)
k_split_x(int64_t ng, const float2 *__restrict__ x, int64_t ld, int64_t ldk, uint32_t *__restrict__ xs_hi,
          uint32_t *__restrict__ xs_lo)
{
    const int b = blockIdx.y;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < ldk; g += (int64_t)gridDim.x * 256) {
        uint32_t hi = 0, lo = 0;
        if (g < ng) {
            const float2 v = x[(size_t)b * ld + g];
            split_pair(v.x, v.y, hi, lo);
        }
        xs_hi[(size_t)b * ldk + g] = hi;
        xs_lo[(size_t)b * ldk + g] = lo;
    }
}

// Wave tile (16 TU) x (16 TW), D k-steps of 16 complex values in the
// register prefetch ring.  64 x 64 tiles with two steps in flight (about
// 190 VGPRs and 190 accumulation registers, one wave per SIMD) against
// 32 x 32 with four, at 512 x 640 x 161235: A^H B 2.0 against 6.7 ms, A B
// 1.75 against 2.9 ms (64 x 32 and 32 x 64 in between): the larger tile
// reuses each loaded operand over more products.
template <int TU_, int TW_, int D_, int SLOTS_> struct BfTile {
    static constexpr int TU = TU_, TW = TW_, D = D_, slots = SLOTS_;
    static constexpr int ring = 16 * D;  // complex k per ring pass
};
using HnTile = BfTile<4, 4, 2, 1024>;
using NnTile = BfTile<4, 4, 2, 1024>;

// partial[s][j][i] = sum over k in split s of conj(A[i][k]) B[j][k], from
// hi / lo pairs (row length lda, ldb); kchunk and Kp are whole ring passes.
template <int TU, int TW, int D>
__global__ void __launch_bounds__(256)
k_gemm_hn_bf16(int M, int N, int64_t Kp, int64_t kchunk, int bm, int bn, int64_t units,
               const uint32_t *__restrict__ Ahi, const uint32_t *__restrict__ Alo, int64_t lda,
               const uint32_t *__restrict__ Bhi, const uint32_t *__restrict__ Blo, int64_t ldb,
               double2 *__restrict__ part)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lk = lane >> 4;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t unit = xcd_index(blockIdx.x, gridDim.x) * 4 + wave; unit < units; unit += nw) {
        const int split = (int)(unit / ((int64_t)bm * bn)), blk = (int)(unit % ((int64_t)bm * bn));
        const int i0 = (blk % bm) * 16 * TU, j0 = (blk / bm) * 16 * TW;
        const int64_t kb = (int64_t)split * kchunk;
        const int64_t ke = kb + kchunk < Kp ? kb + kchunk : Kp;
        f4 re[TU][TW], im[TU][TW];
#pragma unroll
        for (int u = 0; u < TU; ++u)
#pragma unroll
            for (int w = 0; w < TW; ++w) {
                re[u][w] = f4{0, 0, 0, 0};
                im[u][w] = f4{0, 0, 0, 0};
            }
        // rows and columns past M and N read the last valid one (never stored)
        const u4 *pah[TU], *pal[TU], *pbh[TW], *pbl[TW];
#pragma unroll
        for (int u = 0; u < TU; ++u) {
            const int64_t o = (int64_t)min(i0 + 16 * u + l16, M - 1) * lda + kb + 4 * lk;
            pah[u] = reinterpret_cast<const u4 *>(Ahi + o);
            pal[u] = reinterpret_cast<const u4 *>(Alo + o);
        }
#pragma unroll
        for (int w = 0; w < TW; ++w) {
            const int64_t o = (int64_t)min(j0 + 16 * w + l16, N - 1) * ldb + kb + 4 * lk;
            pbh[w] = reinterpret_cast<const u4 *>(Bhi + o);
            pbl[w] = reinterpret_cast<const u4 *>(Blo + o);
        }
        u4 ah[D][TU], al[D][TU], bh[D][TW], bl[D][TW];
        // one k-step = 16 complex = 4 u4 per row
        auto load = [&](int slot, int d) {
#pragma unroll
            for (int u = 0; u < TU; ++u) {
                ah[slot][u] = pah[u][4 * d];
                al[slot][u] = pal[u][4 * d];
            }
#pragma unroll
            for (int w = 0; w < TW; ++w) {
                bh[slot][w] = pbh[w][4 * d];
                bl[slot][w] = pbl[w][4 * d];
            }
        };
        auto step = [&](int slot) {
#pragma unroll
            for (int u = 0; u < TU; ++u) {
                const u4 rh = rot(ah[slot][u]), rl = rot(al[slot][u]);
#pragma unroll
                for (int w = 0; w < TW; ++w) {
                    re[u][w] = mma(ah[slot][u], bh[slot][w], re[u][w]);
                    re[u][w] = mma(ah[slot][u], bl[slot][w], re[u][w]);
                    re[u][w] = mma(al[slot][u], bh[slot][w], re[u][w]);
                    im[u][w] = mma(rh, bh[slot][w], im[u][w]);
                    im[u][w] = mma(rh, bl[slot][w], im[u][w]);
                    im[u][w] = mma(rl, bh[slot][w], im[u][w]);
                }
            }
        };
        const int64_t passes = (ke - kb) / (16 * D);
        if (passes > 0) {
#pragma unroll
            for (int d = 0; d < D - 1; ++d) {
                load(d, d);
                __builtin_amdgcn_sched_barrier(0);
            }
            for (int64_t t = passes; t > 1; --t) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    load((d + D - 1) % D, d + D - 1);
                    step(d);
                }
#pragma unroll
                for (int u = 0; u < TU; ++u) {
                    pah[u] += 4 * D;
                    pal[u] += 4 * D;
                }
#pragma unroll
                for (int w = 0; w < TW; ++w) {
                    pbh[w] += 4 * D;
                    pbl[w] += 4 * D;
                }
            }
            load(D - 1, D - 1);
#pragma unroll
            for (int d = 0; d < D; ++d) step(d);
        }
        double2 *P = part + (size_t)split * M * N;
#pragma unroll
        for (int u = 0; u < TU; ++u)
#pragma unroll
            for (int w = 0; w < TW; ++w)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = i0 + 16 * u + 4 * lk + v, j = j0 + 16 * w + l16;
                    if (i < M && j < N) P[(size_t)j * M + i] = make_double2(re[u][w][v], im[u][w][v]);
                }
    }
}

// Y[j] = d .* sum_s part[s][j] (projector coefficients times the KB
// energies), written as the hi / lo pairs of (Y_r, -Y_i) with row length
// ldy (zero past M); quad_j = sum_i d_i |sum_s part|^2.  The summation
// order is that of the FP32 path's reduce kernel.
__global__ void __launch_bounds__(256)
k_gemm_hn_bf16_reduce(int M, int N, int nsplit, const double2 *__restrict__ part, const double *__restrict__ dscale,
                      uint32_t *__restrict__ yhi, uint32_t *__restrict__ ylo, int ldy, double *__restrict__ quad)
{
    __shared__ double red[4];
    __shared__ double2 grp[4][64];
    const int j = blockIdx.x;
    const int r = threadIdx.x & 63, g = threadIdx.x >> 6;
    double q = 0.0;
    for (int i0 = 0; i0 < ldy; i0 += 64) {
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
        if (g == 0 && i < ldy) {
            uint32_t hi = 0, lo = 0;
            if (i < M) {
                double2 t = grp[0][r];
#pragma unroll
                for (int k = 1; k < 4; ++k) {
                    t.x += grp[k][r].x;
                    t.y += grp[k][r].y;
                }
                const double d = dscale[i];
                q += d * (t.x * t.x + t.y * t.y);
                split_pair((float)(t.x * d), (float)(-t.y * d), hi, lo);
            }
            yhi[(size_t)j * ldy + i] = hi;
            ylo[(size_t)j * ldy + i] = lo;
        }
        __syncthreads();
    }
    if (quad) {
        q = block_sum<256>(q, red);
        if (threadIdx.x == 0) quad[j] = q;
    }
}

// C[n][g] (+)= sum_p beta_p(g) Y[n][p]: matrix-core rows = n (the Y pairs,
// row length ldy), columns = g (the transposed projector pairs, row length
// ldbt); Kp (projectors, padded) whole ring passes.
template <int TU, int TW, int D>
__global__ void __launch_bounds__(256)
k_gemm_nn_bf16(int64_t M, int N, int Kp, int bn, int64_t units, const uint32_t *__restrict__ Bthi,
               const uint32_t *__restrict__ Btlo, int64_t ldbt, const uint32_t *__restrict__ Yhi,
               const uint32_t *__restrict__ Ylo, int64_t ldy, float2 *__restrict__ C, int64_t ldc, int accumulate)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lk = lane >> 4;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t unit = xcd_index(blockIdx.x, gridDim.x) * 4 + wave; unit < units; unit += nw) {
        const int64_t g0 = (unit / bn) * 16 * TW;
        const int n0 = (int)(unit % bn) * 16 * TU;
        f4 re[TU][TW], im[TU][TW];
#pragma unroll
        for (int u = 0; u < TU; ++u)
#pragma unroll
            for (int w = 0; w < TW; ++w) {
                re[u][w] = f4{0, 0, 0, 0};
                im[u][w] = f4{0, 0, 0, 0};
            }
        const u4 *pyh[TU], *pyl[TU], *pbh[TW], *pbl[TW];
#pragma unroll
        for (int u = 0; u < TU; ++u) {
            const int64_t o = (int64_t)min(n0 + 16 * u + l16, N - 1) * ldy + 4 * lk;
            pyh[u] = reinterpret_cast<const u4 *>(Yhi + o);
            pyl[u] = reinterpret_cast<const u4 *>(Ylo + o);
        }
#pragma unroll
        for (int w = 0; w < TW; ++w) {
            const int64_t gg = g0 + 16 * w + l16 < M ? g0 + 16 * w + l16 : M - 1;
            const int64_t o = gg * ldbt + 4 * lk;
            pbh[w] = reinterpret_cast<const u4 *>(Bthi + o);
            pbl[w] = reinterpret_cast<const u4 *>(Btlo + o);
        }
        u4 yh[D][TU], yl[D][TU], bh[D][TW], bl[D][TW];
        auto load = [&](int slot, int d) {
#pragma unroll
            for (int u = 0; u < TU; ++u) {
                yh[slot][u] = pyh[u][4 * d];
                yl[slot][u] = pyl[u][4 * d];
            }
#pragma unroll
            for (int w = 0; w < TW; ++w) {
                bh[slot][w] = pbh[w][4 * d];
                bl[slot][w] = pbl[w][4 * d];
            }
        };
        auto step = [&](int slot) {
#pragma unroll
            for (int u = 0; u < TU; ++u) {
                const u4 rh = rot(yh[slot][u]), rl = rot(yl[slot][u]);
#pragma unroll
                for (int w = 0; w < TW; ++w) {
                    re[u][w] = mma(yh[slot][u], bh[slot][w], re[u][w]);
                    re[u][w] = mma(yh[slot][u], bl[slot][w], re[u][w]);
                    re[u][w] = mma(yl[slot][u], bh[slot][w], re[u][w]);
                    im[u][w] = mma(rh, bh[slot][w], im[u][w]);
                    im[u][w] = mma(rh, bl[slot][w], im[u][w]);
                    im[u][w] = mma(rl, bh[slot][w], im[u][w]);
                }
            }
        };
        const int passes = Kp / (16 * D);
        if (passes > 0) {
#pragma unroll
            for (int d = 0; d < D - 1; ++d) {
                load(d, d);
                __builtin_amdgcn_sched_barrier(0);
            }
            for (int t = passes; t > 1; --t) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    load((d + D - 1) % D, d + D - 1);
                    step(d);
                }
#pragma unroll
                for (int u = 0; u < TU; ++u) {
                    pyh[u] += 4 * D;
                    pyl[u] += 4 * D;
                }
#pragma unroll
                for (int w = 0; w < TW; ++w) {
                    pbh[w] += 4 * D;
                    pbl[w] += 4 * D;
                }
            }
            load(D - 1, D - 1);
#pragma unroll
            for (int d = 0; d < D; ++d) step(d);
        }
#pragma unroll
        for (int u = 0; u < TU; ++u) {
            float2 old[TW][4];
            if (accumulate) {
#pragma unroll
                for (int w = 0; w < TW; ++w)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int n = min(n0 + 16 * u + 4 * lk + v, N - 1);
                        const int64_t g = g0 + 16 * w + l16 < M ? g0 + 16 * w + l16 : M - 1;
                        old[w][v] = C[(int64_t)n * ldc + g];
                    }
            }
#pragma unroll
            for (int w = 0; w < TW; ++w)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int n = n0 + 16 * u + 4 * lk + v;
                    const int64_t g = g0 + 16 * w + l16;
                    float2 r = make_float2(re[u][w][v], im[u][w][v]);
                    if (accumulate) {
                        r.x += old[w][v].x;
                        r.y += old[w][v].y;
                    }
                    if (n < N && g < M) C[(int64_t)n * ldc + g] = r;
                }
        }
    }
}

}  // namespace

int64_t bf16_ldk(int64_t ng) { return (ng + HnTile::ring - 1) / HnTile::ring * HnTile::ring; }
int bf16_ldp(int nproj) { return (nproj + NnTile::ring - 1) / NnTile::ring * NnTile::ring; }

hipError_t launch_split_beta(const Plan &pl)
{
    if (pl.nproj == 0) return hipSuccess;
    const int64_t ldk = pl.bf_ldk;
    const unsigned gx = (unsigned)std::min<int64_t>((ldk + 255) / 256, 4096);
    hipLaunchKernelGGL(k_split_beta, dim3(gx, pl.bf_ldp), dim3(256), 0, pl.stream, pl.ng, pl.nproj, pl.beta, pl.ldv,
                       ldk, pl.bf_ldp, pl.bs_hi, pl.bs_lo, pl.bt_hi, pl.bt_lo);
    return hipGetLastError();
}

size_t bf16_apply_scratch_bytes(const Plan &pl, int nb)
{
    // four arrays, each rounded up to 256 bytes
    return sizeof(uint32_t) * 2 * (size_t)nb * ((size_t)pl.bf_ldk + (size_t)pl.bf_ldp) + 4 * 256;
}

// V_NL x added to out (FP32): x split into hi / lo pairs, P = B^H x on the
// BF16 matrix cores (split-K, FP64 partial sums), Y = D P as pairs, then
// out += B Y.  scratch: bf16_apply_scratch_bytes(pl, nb) bytes.
hipError_t apply_nl_bf16(const Plan &pl, const Workspace &w, int nb, const float2 *x, int64_t ld, float2 *out,
                         int64_t ldo, void *scratch, double *quad)
{
    if (pl.nproj == 0 || nb <= 0) return hipSuccess;
    const int64_t ldk = pl.bf_ldk;
    const int ldp = pl.bf_ldp;
    char *s = static_cast<char *>(scratch);
    auto take = [&](size_t bytes) {
        char *p = s;
        s += (bytes + 255) / 256 * 256;
        return reinterpret_cast<uint32_t *>(p);
    };
    uint32_t *xh = take(sizeof(uint32_t) * nb * ldk), *xl = take(sizeof(uint32_t) * nb * ldk);
    uint32_t *yh = take(sizeof(uint32_t) * nb * ldp), *yl = take(sizeof(uint32_t) * nb * ldp);
    const unsigned gx = (unsigned)std::min<int64_t>((ldk + 255) / 256, 4096);
    hipLaunchKernelGGL(k_split_x, dim3(gx, nb), dim3(256), 0, pl.stream, pl.ng, x, ld, ldk, xh, xl);
    // P = B^H x: as gemm_hn, about one unit per wavefront slot, splits whole ring passes
    {
        constexpr int TU = HnTile::TU, TW = HnTile::TW, D = HnTile::D, ring = HnTile::ring;
        constexpr int64_t slots = HnTile::slots;
        const int M = pl.nproj, N = nb;
        const int bm = (M + 16 * TU - 1) / (16 * TU), bn = (N + 16 * TW - 1) / (16 * TW);
        int64_t nsplit = slots / ((int64_t)bm * bn);
        const int64_t kmax = ldk / ring;
        nsplit = std::max<int64_t>(1, std::min(nsplit, kmax));
        nsplit = std::min<int64_t>(nsplit, (int64_t)(w.part_elems / ((size_t)M * N)));
        if (nsplit < 1) return hipErrorInvalidValue;
        int64_t kchunk = (ldk + nsplit - 1) / nsplit;
        kchunk = (kchunk + ring - 1) / ring * ring;
        nsplit = (ldk + kchunk - 1) / kchunk;
        const int64_t units = (int64_t)bm * bn * nsplit;
        const unsigned wgs = (unsigned)std::min<int64_t>((units + 3) / 4, slots / 4);
        prof_mark(PARO_K_GEMM_HN, pl.stream, true);
        hipLaunchKernelGGL((k_gemm_hn_bf16<TU, TW, D>), dim3(wgs), dim3(256), 0, pl.stream, M, N, ldk, kchunk, bm, bn,
                           units, pl.bs_hi, pl.bs_lo, ldk, xh, xl, ldk, w.part);
        prof_mark(PARO_K_GEMM_HN, pl.stream, false);
        hipLaunchKernelGGL(k_gemm_hn_bf16_reduce, dim3(N), dim3(256), 0, pl.stream, M, N, (int)nsplit, w.part, pl.dkb,
                           yh, yl, ldp, quad);
    }
    // out += B Y
    {
        constexpr int TU = NnTile::TU, TW = NnTile::TW, D = NnTile::D;
        constexpr int64_t slots = NnTile::slots;
        const int64_t M = pl.ng;
        const int N = nb;
        const int bn = (N + 16 * TU - 1) / (16 * TU);
        const int64_t units = (M + 16 * TW - 1) / (16 * TW) * bn;
        const unsigned wgs = (unsigned)std::min<int64_t>((units + 3) / 4, slots / 4);
        prof_mark(PARO_K_GEMM_NN, pl.stream, true);
        hipLaunchKernelGGL((k_gemm_nn_bf16<TU, TW, D>), dim3(wgs), dim3(256), 0, pl.stream, M, N, ldp, bn, units,
                           pl.bt_hi, pl.bt_lo, (int64_t)ldp, yh, yl, (int64_t)ldp, out, ldo, 1);
        prof_mark(PARO_K_GEMM_NN, pl.stream, false);
    }
    return hipGetLastError();
}

}  // namespace paro
