// Batched mixed-radix FFT lines for gfx950, double (double2) or single
// (float2) precision complex.
//
// A line of length N is owned by T consecutive "line threads"; each holds
// E = N / T elements in registers.  The transform is a Stockham autosort
// sequence of radix passes R0, R1, ... (product N).  Inside a pass thread t
// runs E / R radix-R butterflies on tasks j = t + T q; between passes the
// line goes through LDS once (store, barrier, load).  After the last pass
// of radix RL the thread holds output index j + r (N / RL) in v[q RL + r],
// which are exactly the input positions of a pass of radix RL: a forward
// transform that starts with RL can run on the registers an inverse
// transform that ended with RL left behind.
//
// X_k = sum_j x_j exp(SIGN 2 pi i j k / N), unnormalised.
#pragma once
#include <hip/hip_runtime.h>

namespace paro {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// complex value of type C2 (double2 or float2) from two doubles
template <class C2> __device__ __forceinline__ C2 cmk(double x, double y);
template <> __device__ __forceinline__ double2 cmk<double2>(double x, double y) { return make_double2(x, y); }
template <> __device__ __forceinline__ float2 cmk<float2>(double x, double y) { return make_float2((float)x, (float)y); }
template <class C2> using RealOf = decltype(C2{}.x);
// SIGN * i * a
template <int SIGN, class C2> __device__ __forceinline__ C2 mul_si(C2 a)
{
    C2 r;
    if (SIGN > 0) {
        r.x = -a.y;
        r.y = a.x;
    } else {
        r.x = a.y;
        r.y = -a.x;
    }
    return r;
}

// cos / sin (2 pi j / R), j < R, correctly rounded literals.
template <int R> struct TwC;
template <> struct TwC<4> {
    static constexpr double c[4] = {1.0, 0.0, -1.0, 0.0};
    static constexpr double s[4] = {0.0, 1.0, 0.0, -1.0};
};
template <> struct TwC<6> {
    static constexpr double c[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
    static constexpr double s[6] = {0.0, 0.8660254037844386467637, 0.8660254037844386467637, 0.0,
                                    -0.8660254037844386467637, -0.8660254037844386467637};
};
template <> struct TwC<8> {
    static constexpr double c[8] = {1.0, 0.7071067811865475244008, 0.0, -0.7071067811865475244008,
                                    -1.0, -0.7071067811865475244008, 0.0, 0.7071067811865475244008};
    static constexpr double s[8] = {0.0, 0.7071067811865475244008, 1.0, 0.7071067811865475244008,
                                    0.0, -0.7071067811865475244008, -1.0, -0.7071067811865475244008};
};
template <> struct TwC<10> {
    static constexpr double c[10] = {1.0, 0.8090169943749474241023, 0.3090169943749474241023,
                                     -0.3090169943749474241023, -0.8090169943749474241023, -1.0,
                                     -0.8090169943749474241023, -0.3090169943749474241023,
                                     0.3090169943749474241023, 0.8090169943749474241023};
    static constexpr double s[10] = {0.0, 0.5877852522924731291687, 0.9510565162951535721164,
                                     0.9510565162951535721164, 0.5877852522924731291687, 0.0,
                                     -0.5877852522924731291687, -0.9510565162951535721164,
                                     -0.9510565162951535721164, -0.5877852522924731291687};
};
template <> struct TwC<12> {
    static constexpr double c[12] = {1.0, 0.8660254037844386467637, 0.5, 0.0, -0.5,
                                     -0.8660254037844386467637, -1.0, -0.8660254037844386467637,
                                     -0.5, 0.0, 0.5, 0.8660254037844386467637};
    static constexpr double s[12] = {0.0, 0.5, 0.8660254037844386467637, 1.0, 0.8660254037844386467637,
                                     0.5, 0.0, -0.5, -0.8660254037844386467637, -1.0,
                                     -0.8660254037844386467637, -0.5};
};
template <> struct TwC<16> {
    static constexpr double c[16] = {1.0, 0.9238795325112867561282, 0.7071067811865475244008,
                                     0.3826834323650897717285, 0.0, -0.3826834323650897717285,
                                     -0.7071067811865475244008, -0.9238795325112867561282, -1.0,
                                     -0.9238795325112867561282, -0.7071067811865475244008,
                                     -0.3826834323650897717285, 0.0, 0.3826834323650897717285,
                                     0.7071067811865475244008, 0.9238795325112867561282};
    static constexpr double s[16] = {0.0, 0.3826834323650897717285, 0.7071067811865475244008,
                                     0.9238795325112867561282, 1.0, 0.9238795325112867561282,
                                     0.7071067811865475244008, 0.3826834323650897717285, 0.0,
                                     -0.3826834323650897717285, -0.7071067811865475244008,
                                     -0.9238795325112867561282, -1.0, -0.9238795325112867561282,
                                     -0.7071067811865475244008, -0.3826834323650897717285};
};
template <> struct TwC<20> {
    static constexpr double c[20] = {1.0, 0.9510565162951535721164, 0.8090169943749474241023,
                                     0.5877852522924731291687, 0.3090169943749474241023, 0.0,
                                     -0.3090169943749474241023, -0.5877852522924731291687,
                                     -0.8090169943749474241023, -0.9510565162951535721164, -1.0,
                                     -0.9510565162951535721164, -0.8090169943749474241023,
                                     -0.5877852522924731291687, -0.3090169943749474241023, 0.0,
                                     0.3090169943749474241023, 0.5877852522924731291687,
                                     0.8090169943749474241023, 0.9510565162951535721164};
    static constexpr double s[20] = {0.0, 0.3090169943749474241023, 0.5877852522924731291687,
                                     0.8090169943749474241023, 0.9510565162951535721164, 1.0,
                                     0.9510565162951535721164, 0.8090169943749474241023,
                                     0.5877852522924731291687, 0.3090169943749474241023, 0.0,
                                     -0.3090169943749474241023, -0.5877852522924731291687,
                                     -0.8090169943749474241023, -0.9510565162951535721164, -1.0,
                                     -0.9510565162951535721164, -0.8090169943749474241023,
                                     -0.5877852522924731291687, -0.3090169943749474241023};
};

// ---------------------------------------------------------------- radix-R DFTs
// Dft<R, SIGN>::run(v): in-place R-point DFT of v[0..R) (double2 or float2).
template <int R, int SIGN> struct Dft;

template <int SIGN> struct Dft<1, SIGN> {
    template <class C2> static __device__ __forceinline__ void run(C2 *) {}
};

template <int SIGN> struct Dft<2, SIGN> {
    template <class C2> static __device__ __forceinline__ void run(C2 *v)
    {
        C2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <int SIGN> struct Dft<3, SIGN> {
    template <class C2> static __device__ __forceinline__ void run(C2 *v)
    {
        using S = RealOf<C2>;
        const S h = (S)0.8660254037844386467637;  // sin(2 pi / 3)
        C2 t1 = cadd(v[1], v[2]);
        C2 t2;
        t2.x = v[0].x - (S)0.5 * t1.x;
        t2.y = v[0].y - (S)0.5 * t1.y;
        C2 t3 = cscale(csub(v[1], v[2]), h);
        C2 it3 = mul_si<SIGN>(t3);
        v[0] = cadd(v[0], t1);
        v[1] = cadd(t2, it3);
        v[2] = csub(t2, it3);
    }
};

template <int SIGN> struct Dft<4, SIGN> {
    template <class C2> static __device__ __forceinline__ void run(C2 *v)
    {
        C2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
        C2 c = cadd(v[1], v[3]), d = mul_si<SIGN>(csub(v[1], v[3]));
        v[0] = cadd(a, c);
        v[2] = csub(a, c);
        v[1] = cadd(b, d);
        v[3] = csub(b, d);
    }
};

template <int SIGN> struct Dft<5, SIGN> {
    template <class C2> static __device__ __forceinline__ void run(C2 *v)
    {
        using S = RealOf<C2>;
        const S c1 = (S)0.3090169943749474241023, c2 = (S)-0.8090169943749474241023;
        const S s1 = (S)0.9510565162951535721164, s2 = (S)0.5877852522924731291687;
        C2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
        C2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
        C2 x0 = v[0];
        C2 p1, p2, q1, q2;
        p1.x = x0.x + c1 * a1.x + c2 * a2.x;
        p1.y = x0.y + c1 * a1.y + c2 * a2.y;
        p2.x = x0.x + c2 * a1.x + c1 * a2.x;
        p2.y = x0.y + c2 * a1.y + c1 * a2.y;
        q1.x = s1 * b1.x + s2 * b2.x;
        q1.y = s1 * b1.y + s2 * b2.y;
        q2.x = s2 * b1.x - s1 * b2.x;
        q2.y = s2 * b1.y - s1 * b2.y;
        q1 = mul_si<SIGN>(q1);
        q2 = mul_si<SIGN>(q2);
        v[0] = cadd(x0, cadd(a1, a2));
        v[1] = cadd(p1, q1);
        v[4] = csub(p1, q1);
        v[2] = cadd(p2, q2);
        v[3] = csub(p2, q2);
    }
};

// R = A B: A-point DFTs over s_a of x[B s_a + s_b], twiddle by w_R^(s_b k_a),
// then B-point DFTs over s_b; output index k_a + A k_b.
template <int A, int B, int SIGN> struct DftComp {
    template <class C2> static __device__ __forceinline__ void run(C2 *v)
    {
        using S = RealOf<C2>;
        constexpr int R = A * B;
        C2 y[R];
#pragma unroll
        for (int sb = 0; sb < B; ++sb) {
            C2 a[A];
#pragma unroll
            for (int sa = 0; sa < A; ++sa) a[sa] = v[B * sa + sb];
            Dft<A, SIGN>::run(a);
#pragma unroll
            for (int ka = 0; ka < A; ++ka) y[sb * A + ka] = a[ka];
        }
#pragma unroll
        for (int ka = 0; ka < A; ++ka) {
            C2 b[B];
#pragma unroll
            for (int sb = 0; sb < B; ++sb) {
                const int j = sb * ka;
                C2 x = y[sb * A + ka];
                if (j != 0) {
                    const S c = (S)TwC<R>::c[j], s = (S)(SIGN * TwC<R>::s[j]);
                    C2 t;
                    t.x = x.x * c - x.y * s;
                    t.y = x.x * s + x.y * c;
                    x = t;
                }
                b[sb] = x;
            }
            Dft<B, SIGN>::run(b);
#pragma unroll
            for (int kb = 0; kb < B; ++kb) v[ka + A * kb] = b[kb];
        }
    }
};

template <int SIGN> struct Dft<6, SIGN> : DftComp<2, 3, SIGN> {};
template <int SIGN> struct Dft<8, SIGN> : DftComp<2, 4, SIGN> {};
template <int SIGN> struct Dft<10, SIGN> : DftComp<2, 5, SIGN> {};
template <int SIGN> struct Dft<12, SIGN> : DftComp<4, 3, SIGN> {};
template <int SIGN> struct Dft<16, SIGN> : DftComp<4, 4, SIGN> {};
template <int SIGN> struct Dft<20, SIGN> : DftComp<4, 5, SIGN> {};

// ---------------------------------------------------------------- line schedules
template <int... Rs> struct RList {};

template <int First, int... Rest> struct FirstOf { static constexpr int value = First; };
template <int... Rs> struct LastOf;
template <int R> struct LastOf<R> { static constexpr int value = R; };
template <int R, int... Rs> struct LastOf<R, Rs...> { static constexpr int value = LastOf<Rs...>::value; };

// FftCfg<N>: T threads per line, E = N / T elements each, radix list Inv
// (used for SIGN = +1) and its reverse Fwd (SIGN = -1).
template <int N> struct FftCfg;
template <> struct FftCfg<8> { static constexpr int N = 8, T = 2, E = 4; using Inv = RList<4, 2>; using Fwd = RList<2, 4>; };
template <> struct FftCfg<16> { static constexpr int N = 16, T = 4, E = 4; using Inv = RList<4, 4>; using Fwd = RList<4, 4>; };
template <> struct FftCfg<24> { static constexpr int N = 24, T = 2, E = 12; using Inv = RList<6, 4>; using Fwd = RList<4, 6>; };
template <> struct FftCfg<32> { static constexpr int N = 32, T = 4, E = 8; using Inv = RList<8, 4>; using Fwd = RList<4, 8>; };
template <> struct FftCfg<40> { static constexpr int N = 40, T = 2, E = 20; using Inv = RList<10, 4>; using Fwd = RList<4, 10>; };
template <> struct FftCfg<48> { static constexpr int N = 48, T = 4, E = 12; using Inv = RList<12, 4>; using Fwd = RList<4, 12>; };
template <> struct FftCfg<64> { static constexpr int N = 64, T = 8, E = 8; using Inv = RList<8, 8>; using Fwd = RList<8, 8>; };
template <> struct FftCfg<80> { static constexpr int N = 80, T = 4, E = 20; using Inv = RList<5, 4, 4>; using Fwd = RList<4, 4, 5>; };
template <> struct FftCfg<96> { static constexpr int N = 96, T = 8, E = 12; using Inv = RList<6, 4, 4>; using Fwd = RList<4, 4, 6>; };
template <> struct FftCfg<160> { static constexpr int N = 160, T = 8, E = 20; using Inv = RList<10, 4, 4>; using Fwd = RList<4, 4, 10>; };

template <class L> struct ListInfo;
template <int... Rs> struct ListInfo<RList<Rs...>> {
    static constexpr int first = FirstOf<Rs...>::value;
    static constexpr int last = LastOf<Rs...>::value;
};

// Inputs of a radix-R pass: v[q R + r] <- x[t + T q + r N/R].
template <int N, int T, int E, int R, class C2, class F>
__device__ __forceinline__ void pass_load(C2 (&v)[E], int t, F &&f)
{
#pragma unroll
    for (int q = 0; q < E / R; ++q)
#pragma unroll
        for (int r = 0; r < R; ++r) v[q * R + r] = f(t + T * q + r * (N / R));
}

// Outputs of a radix-R pass at stride NS: v[q R + r] -> y[(j/NS) NS R + j%NS + r NS].
template <int N, int T, int E, int R, int NS, class C2, class F>
__device__ __forceinline__ void pass_store(const C2 (&v)[E], int t, F &&f)
{
#pragma unroll
    for (int q = 0; q < E / R; ++q) {
        const int j = t + T * q;
        const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int r = 0; r < R; ++r) f(base + r * NS, v[q * R + r]);
    }
}

// Final outputs (after a last pass of radix RL): v[q RL + r] is element t + T q + r N/RL.
template <int N, int T, int E, int RL, class C2, class F>
__device__ __forceinline__ void final_foreach(const C2 (&v)[E], int t, F &&f)
{
#pragma unroll
    for (int q = 0; q < E / RL; ++q)
#pragma unroll
        for (int r = 0; r < RL; ++r) f(t + T * q + r * (N / RL), q * RL + r);
}

// tw[m] = exp(-2 pi i m / N) (same precision as v); SIGN = +1 uses the conjugate.
template <int N, int T, int E, int R, int NS, int SIGN, class C2>
__device__ __forceinline__ void pass_compute(C2 (&v)[E], int t, const C2 *__restrict__ tw)
{
#pragma unroll
    for (int q = 0; q < E / R; ++q) {
        if constexpr (NS > 1) {
            const int j = t + T * q;
            const int k = j % NS;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                C2 w = tw[r * k * (N / (NS * R))];
                if (SIGN > 0) w.y = -w.y;
                v[q * R + r] = cmul(v[q * R + r], w);
            }
        }
        Dft<R, SIGN>::run(&v[q * R]);
    }
}

// Order LDS accesses between the lanes of one wavefront: every line of a
// transform lives inside one wavefront (T divides 64 and line threads are
// consecutive lanes), so exchanges between passes need no work-group
// barrier.  LDS operations of a wavefront complete in order; the wait and
// the fences keep the compiler from moving loads above the stores.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool WL> __device__ __forceinline__ void line_sync()
{
    if constexpr (WL) wave_lds_sync();
    else __syncthreads();
}

template <int N, int T, int E, int SIGN, bool WL, int NS, int R, int... Rest, class C2>
__device__ __forceinline__ void stockham_rec(C2 (&v)[E], int t, bool act, C2 *line, int es, const C2 *tw)
{
    // An opaque zero offset per pass keeps the compiler from loading the
    // twiddles of later passes (or other transforms) up front, which costs
    // registers; without work-group barriers nothing else bounds that code
    // motion.  The offset, not the pointer, is made opaque: the pointer keeps
    // its address space, so the reads stay global or LDS reads (a flat read
    // would also hold up every LDS wait of the exchanges).
    if constexpr (NS > 1) {
        int zero = 0;
        asm volatile("" : "+s"(zero));
        tw += zero;
    }
    if (act) pass_compute<N, T, E, R, NS, SIGN>(v, t, tw);
    if constexpr (sizeof...(Rest) > 0) {
        constexpr int R2 = FirstOf<Rest...>::value;
        line_sync<WL>();
        if (act) pass_store<N, T, E, R, NS>(v, t, [&](int i, C2 x) { line[i * es] = x; });
        line_sync<WL>();
        if (act) pass_load<N, T, E, R2>(v, t, [&](int i) { return line[i * es]; });
        stockham_rec<N, T, E, SIGN, WL, NS * R, Rest...>(v, t, act, line, es, tw);
    }
}

// Run all passes of list L on registers v that hold the inputs of its first
// pass, for a line schedule Cfg (N, T threads per line, E elements each).
// line/es: this thread's line in LDS, used for the exchanges between
// passes.  WL = false: every thread of the block must call this (it
// contains work-group barriers; act = false threads only take part in
// them).  WL = true: the T threads of each line are consecutive lanes of one
// wavefront and only wavefront-level ordering is used.
template <class Cfg, int SIGN, bool WL = false, int... Rs, class C2>
__device__ __forceinline__ void stockham_c(RList<Rs...>, C2 (&v)[Cfg::E], int t, bool act, C2 *line, int es,
                                           const C2 *__restrict__ tw)
{
    static_assert(!WL || 64 % Cfg::T == 0, "wave-local lines need T | 64");
    int zero = 0;
    asm volatile("" : "+s"(zero));
    stockham_rec<Cfg::N, Cfg::T, Cfg::E, SIGN, WL, 1, Rs...>(v, t, act, line, es, tw + zero);
}

template <int N, int SIGN, bool WL = false, int... Rs, class C2>
__device__ __forceinline__ void stockham(RList<Rs...> l, C2 (&v)[FftCfg<N>::E], int t, bool act, C2 *line, int es,
                                         const C2 *__restrict__ tw)
{
    stockham_c<FftCfg<N>, SIGN, WL>(l, v, t, act, line, es, tw);
}

// ---------------------------------------------------------------------------
// 96-point transform of one line across 8 lanes without LDS (FP64 or FP32).
//
// Thread t of the line (lane bits 3, 4, 5 = bits 0, 1, 2 of t) holds
// x[t + 8 m], m < 12.  Four-step split 96 = 12 x 8: a 12-point DFT over m in
// registers, the twiddle w^(t k1), then 8-point DFTs over t across the lanes
// as three radix-2 decimation-in-frequency stages on thread bits 2, 1, 0
// (lane distances 32, 16, 8).  Each stage first swaps half of the twelve
// registers with the partner lane (v_permlane32_swap / v_permlane16_swap,
// or two DPP row rotations for distance 8), so that each lane then holds
// both operands of six butterflies.  After the three stages register s of
// thread t holds X[k] with, for s = j + 3 d + 6 e (j < 3, d, e < 2),
// k = (j + 3 t1 + 6 t2) + 12 (4 e + 2 d + t0), t = t0 + 2 t1 + 4 t2
// (xlane_index).  The forward transform applies the conjugate transpose of
// every step in reverse order, so its outputs are again x[t + 8 m].
__host__ __device__ constexpr int xlane_index(int t, int s)
{
    return (s % 3 + 3 * (t >> 1 & 1) + 6 * (t >> 2 & 1)) + 12 * (4 * (s / 6) + 2 * (s / 3 % 2) + (t & 1));
}

__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// Lane swap on thread bit B: the line's lower lane (bit B clear) receives
// the upper lane's p in q, the upper lane receives the lower lane's q in p.
template <int B> __device__ __forceinline__ void xswap32(uint32_t &p, uint32_t &q);
template <> __device__ __forceinline__ void xswap32<2>(uint32_t &p, uint32_t &q)
{
    const auto r = __builtin_amdgcn_permlane32_swap(p, q, false, false);
    p = r[0];
    q = r[1];
}
template <> __device__ __forceinline__ void xswap32<1>(uint32_t &p, uint32_t &q)
{
    const auto r = __builtin_amdgcn_permlane16_swap(p, q, false, false);
    p = r[0];
    q = r[1];
}
template <> __device__ __forceinline__ void xswap32<0>(uint32_t &p, uint32_t &q)
{
    // row_ror:8 pairs lanes l and l ^ 8 of each 16-lane row; banks 0-1 of
    // a row are its lanes 0-7 (thread bit 0 clear), banks 2-3 lanes 8-15
    const int p0 = (int)p, q0 = (int)q;
    q = (uint32_t)__builtin_amdgcn_update_dpp(q0, p0, 0x128, 0xf, 0x3, false);
    p = (uint32_t)__builtin_amdgcn_update_dpp(p0, q0, 0x128, 0xf, 0xc, false);
}
template <int B, class C2> __device__ __forceinline__ void xswap(C2 &p, C2 &q)
{
    constexpr int W = sizeof(C2) / 4;  // 32-bit words per complex value
    uint32_t a[W], b[W];
    __builtin_memcpy(a, &p, sizeof(C2));
    __builtin_memcpy(b, &q, sizeof(C2));
#pragma unroll
    for (int i = 0; i < W; ++i) xswap32<B>(a[i], b[i]);
    __builtin_memcpy(&p, a, sizeof(C2));
    __builtin_memcpy(&q, b, sizeof(C2));
}

// register pairs of the butterflies of the stage on thread bit B
template <int B> __device__ __forceinline__ constexpr int xpair_lo(int i)
{
    return B == 1 ? (i % 3) + 6 * (i / 3) : i;
}
template <int B> __device__ __forceinline__ constexpr int xpair_hi(int i)
{
    return B == 1 ? (i % 3) + 3 + 6 * (i / 3) : i + 6;
}

// inverse-direction stage: swap, then (u, v) -> (u + v, (u - v) w)
// (W false: w is 1 and the multiply is left out)
template <int B, bool W = true, class C2> __device__ __forceinline__ void xstage_inv(C2 (&v)[12], C2 w)
{
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        C2 &a = v[xpair_lo<B>(i)], &b = v[xpair_hi<B>(i)];
        xswap<B>(a, b);
        const C2 u = a, d = csub(a, b);
        a = cadd(u, b);
        b = (B == 0 || !W) ? d : cmul(d, w);
    }
}
// its conjugate transpose: (a, b) -> (a + b w*, a - b w*), then the same swap
template <int B, bool W = true, class C2> __device__ __forceinline__ void xstage_fwd(C2 (&v)[12], C2 wc)
{
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        C2 &a = v[xpair_lo<B>(i)], &b = v[xpair_hi<B>(i)];
        const C2 c = (B == 0 || !W) ? b : cmul(b, wc);
        const C2 u = a;
        a = cadd(u, c);
        b = csub(u, c);
        xswap<B>(a, b);
    }
}

// tw[m] = exp(-2 pi i m / 96), an LDS copy of the plan's table: every
// transform reads 13 twiddles, and through the vector memory path these
// loads cost more than the arithmetic around them.  Callers pass t through
// an opaque copy at each call, so that the compiler does not hoist the
// twiddle reads of one call site into registers across the others.
// Inverse: v[m] = x[t + 8 m] on entry, v[s] = X[xlane_index(t, s)] (sign
// +1, unnormalised) on exit.
// Pruned 12-point DFTs (the DftComp<4, 3> order of Dft<12>) for lines whose
// populated indices all lie within |n| <= 23, so that x[t + 8 m] is zero
// for m = 3..8 on input and those outputs are never used.  Every output
// that is computed comes from the same floating-point operations as in
// Dft<12>, less additions of exact zeros and with a subtraction in place of
// adding a negation, so the values agree with the full transform's (up to
// the sign of an exact zero).
__host__ __device__ constexpr bool xlane_kept(int m) { return m < 3 || m > 8; }

template <int SIGN, class C2> __device__ __forceinline__ void dft12_twiddle(C2 (&b)[3], int ka)
{
    using S = RealOf<C2>;
#pragma unroll
    for (int sb = 1; sb < 3; ++sb) {
        const int j = sb * ka;
        if (j != 0) {
            const S c = (S)TwC<12>::c[j], sn = (S)(SIGN * TwC<12>::s[j]);
            C2 r;
            r.x = b[sb].x * c - b[sb].y * sn;
            r.y = b[sb].x * sn + b[sb].y * c;
            b[sb] = r;
        }
    }
}
// inputs 3..8 zero: the 4-point DFTs over s_a see only s_a = 0 and 3
template <int SIGN, class C2> __device__ __forceinline__ void dft12_in_pruned(C2 (&v)[12])
{
    C2 y[12];
#pragma unroll
    for (int sb = 0; sb < 3; ++sb) {
        const C2 a0 = v[sb], a3 = v[9 + sb];
        const C2 d = mul_si<SIGN>(a3);
        y[sb * 4 + 0] = cadd(a0, a3);
        y[sb * 4 + 2] = csub(a0, a3);
        y[sb * 4 + 1] = csub(a0, d);
        y[sb * 4 + 3] = cadd(a0, d);
    }
#pragma unroll
    for (int ka = 0; ka < 4; ++ka) {
        C2 b[3] = {y[ka], y[4 + ka], y[8 + ka]};
        dft12_twiddle<SIGN>(b, ka);
        Dft<3, SIGN>::run(b);
#pragma unroll
        for (int kb = 0; kb < 3; ++kb) v[ka + 4 * kb] = b[kb];
    }
}
// outputs 3..8 unused: of the 3-point DFTs only the outputs k_a + 4 k_b
// with k = 0, 1, 2, 9, 10, 11 are formed (outputs 3..8 are left undefined)
template <int SIGN, class C2> __device__ __forceinline__ void dft12_out_pruned(C2 (&v)[12])
{
    using S = RealOf<C2>;
    C2 y[12];
#pragma unroll
    for (int sb = 0; sb < 3; ++sb) {
        C2 a[4] = {v[sb], v[3 + sb], v[6 + sb], v[9 + sb]};
        Dft<4, SIGN>::run(a);
#pragma unroll
        for (int ka = 0; ka < 4; ++ka) y[sb * 4 + ka] = a[ka];
    }
#pragma unroll
    for (int ka = 0; ka < 4; ++ka) {
        C2 b[3] = {y[ka], y[4 + ka], y[8 + ka]};
        dft12_twiddle<SIGN>(b, ka);
        // the operations of Dft<3> for the outputs that are needed
        const S h = (S)0.8660254037844386467637;  // sin(2 pi / 3)
        const C2 t1 = cadd(b[1], b[2]);
        if (ka < 3) v[ka] = cadd(b[0], t1);  // k_b = 0
        if (ka > 0) {                          // k_b = 2
            C2 t2;
            t2.x = b[0].x - (S)0.5 * t1.x;
            t2.y = b[0].y - (S)0.5 * t1.y;
            const C2 it3 = mul_si<SIGN>(cscale(csub(b[1], b[2]), h));
            v[ka + 8] = csub(t2, it3);
        }
    }
}

template <bool PRUNE = false, class C2>
__device__ __forceinline__ void xlane96_inverse(C2 (&v)[12], int t, const C2 *__restrict__ tw)
{
    if constexpr (PRUNE) dft12_in_pruned<+1>(v);
    else Dft<12, +1>::run(v);
#pragma unroll
    for (int k = 1; k < 12; ++k) v[k] = cmul(v[k], cconj(tw[t * k]));
    xstage_inv<2>(v, cconj(tw[12 * (t & 3)]));
    xstage_inv<1>(v, cconj(tw[24 * (t & 1)]));
    xstage_inv<0>(v, cmk<C2>(1.0, 0.0));
}
// Forward (sign -1) from the layout xlane96_inverse leaves: v[m] = y[t + 8 m] on exit.
template <bool PRUNE = false, class C2>
__device__ __forceinline__ void xlane96_forward(C2 (&v)[12], int t, const C2 *__restrict__ tw)
{
    xstage_fwd<0>(v, cmk<C2>(1.0, 0.0));
    xstage_fwd<1>(v, tw[24 * (t & 1)]);
    xstage_fwd<2>(v, tw[12 * (t & 3)]);
#pragma unroll
    for (int k = 1; k < 12; ++k) v[k] = cmul(v[k], tw[t * k]);
    if constexpr (PRUNE) dft12_out_pruned<-1>(v);
    else Dft<12, -1>::run(v);
}

// The same 96-point schedule with two of its threads in each lane: a line
// takes four lanes u = 0..3 (lane distances 16 and 32, the swaps of thread
// bits 1 and 2), and lane u holds the registers of threads 2 u (set a) and
// 2 u + 1 (set b).  The 12-point DFTs, the twiddles and the stages on
// thread bits 2 and 1 are those of xlane96_inverse, once per set; the stage
// on thread bit 0 pairs the two sets inside the lane, where the swap
// becomes a renaming of registers (no exchange at all).  Thread 2 u has
// the stage-1 twiddle 1, so that multiply is left out.  On exit register
// s of set j holds X[xlane_index(2 u + j, s)], as thread 2 u + j of the
// eight-lane schedule would.
template <class C2> __device__ __forceinline__ void xstage_inv_bit0(C2 (&a)[12], C2 (&b)[12])
{
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        // after the eight-lane swap thread 2 u would hold (a[i], b[i]) and
        // thread 2 u + 1 (a[i + 6], b[i + 6]) in its registers i and i + 6
        const C2 pa = a[i], qa = b[i], pb = a[i + 6], qb = b[i + 6];
        a[i] = cadd(pa, qa);
        a[i + 6] = csub(pa, qa);
        b[i] = cadd(pb, qb);
        b[i + 6] = csub(pb, qb);
    }
}
template <class C2> __device__ __forceinline__ void xstage_fwd_bit0(C2 (&a)[12], C2 (&b)[12])
{
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const C2 sa = cadd(a[i], a[i + 6]), da = csub(a[i], a[i + 6]);
        const C2 sb = cadd(b[i], b[i + 6]), db = csub(b[i], b[i + 6]);
        // the swap: thread 2 u keeps its sum and receives the other's; the
        // differences go to thread 2 u + 1
        a[i] = sa;
        a[i + 6] = sb;
        b[i] = da;
        b[i + 6] = db;
    }
}
template <bool PRUNE = false, class C2>
__device__ __forceinline__ void xlane96x2_inverse(C2 (&a)[12], C2 (&b)[12], int u, const C2 *__restrict__ tw)
{
    const int ta = 2 * u, tb = ta + 1;
    if constexpr (PRUNE) {
        dft12_in_pruned<+1>(a);
        dft12_in_pruned<+1>(b);
    } else {
        Dft<12, +1>::run(a);
        Dft<12, +1>::run(b);
    }
#pragma unroll
    for (int k = 1; k < 12; ++k) {
        a[k] = cmul(a[k], cconj(tw[ta * k]));
        b[k] = cmul(b[k], cconj(tw[tb * k]));
    }
    xstage_inv<2>(a, cconj(tw[12 * (ta & 3)]));
    xstage_inv<2>(b, cconj(tw[12 * (tb & 3)]));
    xstage_inv<1, false>(a, cmk<C2>(1.0, 0.0));
    xstage_inv<1>(b, cconj(tw[24]));
    xstage_inv_bit0(a, b);
}
// Forward (sign -1) from the layout xlane96x2_inverse leaves: a[m] =
// y[2 u + 8 m], b[m] = y[2 u + 1 + 8 m] on exit.
template <bool PRUNE = false, class C2>
__device__ __forceinline__ void xlane96x2_forward(C2 (&a)[12], C2 (&b)[12], int u, const C2 *__restrict__ tw)
{
    const int ta = 2 * u, tb = ta + 1;
    xstage_fwd_bit0(a, b);
    xstage_fwd<1, false>(a, cmk<C2>(1.0, 0.0));
    xstage_fwd<1>(b, tw[24]);
    xstage_fwd<2>(a, tw[12 * (ta & 3)]);
    xstage_fwd<2>(b, tw[12 * (tb & 3)]);
#pragma unroll
    for (int k = 1; k < 12; ++k) {
        a[k] = cmul(a[k], tw[ta * k]);
        b[k] = cmul(b[k], tw[tb * k]);
    }
    if constexpr (PRUNE) {
        dft12_out_pruned<-1>(a);
        dft12_out_pruned<-1>(b);
    } else {
        Dft<12, -1>::run(a);
        Dft<12, -1>::run(b);
    }
}

// The same schedule for any N = 8 E with E = 4 J (160 points: E = 20, a
// 20-point DFT in registers).  Register s = j + J d + 2 J e (j < J, d, e <
// 2); the stages pair registers (i, i + 2 J) on thread bits 2 and 0 and
// (j + 2 J c, j + J + 2 J c) on bit 1, and after the three stages register s
// of thread t holds X[k] with
// k = (j + J t1 + 2 J t2) + E (4 e + 2 d + t0) (xlane_index_e); for E = 12
// these are the pairs and the order of the 96-point functions above.
template <int E> __host__ __device__ constexpr int xlane_index_e(int t, int s)
{
    constexpr int J = E / 4;
    return (s % J + J * (t >> 1 & 1) + 2 * J * (t >> 2 & 1)) + E * (4 * (s / (2 * J)) + 2 * (s / J % 2) + (t & 1));
}
template <int B, int E> __device__ __forceinline__ constexpr int xpair_lo_e(int i)
{
    constexpr int J = E / 4;
    return B == 1 ? (i % J) + 2 * J * (i / J) : i;
}
template <int B, int E> __device__ __forceinline__ constexpr int xpair_hi_e(int i)
{
    constexpr int J = E / 4;
    return B == 1 ? (i % J) + J + 2 * J * (i / J) : i + 2 * J;
}
template <int B, int E, class C2> __device__ __forceinline__ void xstage_inv_e(C2 (&v)[E], C2 w)
{
#pragma unroll
    for (int i = 0; i < E / 2; ++i) {
        C2 &a = v[xpair_lo_e<B, E>(i)], &b = v[xpair_hi_e<B, E>(i)];
        xswap<B>(a, b);
        const C2 u = a, d = csub(a, b);
        a = cadd(u, b);
        b = B == 0 ? d : cmul(d, w);
    }
}
template <int B, int E, class C2> __device__ __forceinline__ void xstage_fwd_e(C2 (&v)[E], C2 wc)
{
#pragma unroll
    for (int i = 0; i < E / 2; ++i) {
        C2 &a = v[xpair_lo_e<B, E>(i)], &b = v[xpair_hi_e<B, E>(i)];
        const C2 c = B == 0 ? b : cmul(b, wc);
        const C2 u = a;
        a = cadd(u, c);
        b = csub(u, c);
        xswap<B>(a, b);
    }
}
// Pruned E-point DFTs for E = 4 B (the DftComp<4, B> order of Dft<E>), the
// generalisation of the 12-point ones above.  A line whose populated
// indices satisfy |n| < 2 E (|n| <= 39 at 160 points, which every plan
// with N >= 4 n_max + 1 meets) holds zeros in x[t + 8 m] for
// E / 4 <= m < 3 E / 4: the inputs B .. 3 B - 1, i.e. s_a = 1 and 2 of the
// 4-point DFTs over x[B s_a + s_b].  Those outputs are never used either.
template <int E> __host__ __device__ constexpr bool xlane_kept_e(int m) { return m < E / 4 || m >= 3 * E / 4; }

template <int B, int SIGN, class C2> __device__ __forceinline__ void dft4b_twiddle(C2 (&b)[B], int ka)
{
    using S = RealOf<C2>;
#pragma unroll
    for (int sb = 1; sb < B; ++sb) {
        const int j = sb * ka;
        if (j != 0) {
            const S c = (S)TwC<4 * B>::c[j], sn = (S)(SIGN * TwC<4 * B>::s[j]);
            C2 r;
            r.x = b[sb].x * c - b[sb].y * sn;
            r.y = b[sb].x * sn + b[sb].y * c;
            b[sb] = r;
        }
    }
}
// inputs B .. 3 B - 1 zero: each 4-point DFT sees only s_a = 0 and 3
template <int B, int SIGN, class C2> __device__ __forceinline__ void dft4b_in_pruned(C2 (&v)[4 * B])
{
    C2 y[4 * B];
#pragma unroll
    for (int sb = 0; sb < B; ++sb) {
        const C2 a0 = v[sb], a3 = v[3 * B + sb];
        const C2 d = mul_si<SIGN>(a3);
        y[sb * 4 + 0] = cadd(a0, a3);
        y[sb * 4 + 2] = csub(a0, a3);
        y[sb * 4 + 1] = csub(a0, d);
        y[sb * 4 + 3] = cadd(a0, d);
    }
#pragma unroll
    for (int ka = 0; ka < 4; ++ka) {
        C2 b[B];
#pragma unroll
        for (int sb = 0; sb < B; ++sb) b[sb] = y[sb * 4 + ka];
        dft4b_twiddle<B, SIGN>(b, ka);
        Dft<B, SIGN>::run(b);
#pragma unroll
        for (int kb = 0; kb < B; ++kb) v[ka + 4 * kb] = b[kb];
    }
}
// outputs B .. 3 B - 1 unused: only the kept outputs are stored (the
// B-point DFTs' other outputs are dead code; the unkept v[k] keep stale values)
template <int B, int SIGN, class C2> __device__ __forceinline__ void dft4b_out_pruned(C2 (&v)[4 * B])
{
    C2 y[4 * B];
#pragma unroll
    for (int sb = 0; sb < B; ++sb) {
        C2 a[4] = {v[sb], v[B + sb], v[2 * B + sb], v[3 * B + sb]};
        Dft<4, SIGN>::run(a);
#pragma unroll
        for (int ka = 0; ka < 4; ++ka) y[sb * 4 + ka] = a[ka];
    }
#pragma unroll
    for (int ka = 0; ka < 4; ++ka) {
        C2 b[B];
#pragma unroll
        for (int sb = 0; sb < B; ++sb) b[sb] = y[sb * 4 + ka];
        dft4b_twiddle<B, SIGN>(b, ka);
        Dft<B, SIGN>::run(b);
#pragma unroll
        for (int kb = 0; kb < B; ++kb)
            if (xlane_kept_e<4 * B>(ka + 4 * kb)) v[ka + 4 * kb] = b[kb];
    }
}

// tw[m] = exp(-2 pi i m / N).  Inverse: v[m] = x[t + 8 m] on entry,
// v[s] = X[xlane_index_e<N / 8>(t, s)] (sign +1, unnormalised) on exit.
// PRUNE: inputs x[t + 8 m] with m not xlane_kept_e are zero (not read).
template <int N, bool PRUNE = false, class C2>
__device__ __forceinline__ void xlane_inverse_n(C2 (&v)[N / 8], int t, const C2 *__restrict__ tw)
{
    constexpr int E = N / 8;
    static_assert(E % 4 == 0, "N = 8 E with E a multiple of 4");
    if constexpr (PRUNE) dft4b_in_pruned<E / 4, +1>(v);
    else Dft<E, +1>::run(v);
#pragma unroll
    for (int k = 1; k < E; ++k) v[k] = cmul(v[k], cconj(tw[t * k]));
    xstage_inv_e<2, E>(v, cconj(tw[(N / 8) * (t & 3)]));
    xstage_inv_e<1, E>(v, cconj(tw[(N / 4) * (t & 1)]));
    xstage_inv_e<0, E>(v, cmk<C2>(1.0, 0.0));
}
// Forward (sign -1) from the layout xlane_inverse_n leaves: v[m] = y[t + 8 m] on exit.
// PRUNE: only the outputs with xlane_kept_e(m) are formed.
template <int N, bool PRUNE = false, class C2>
__device__ __forceinline__ void xlane_forward_n(C2 (&v)[N / 8], int t, const C2 *__restrict__ tw)
{
    constexpr int E = N / 8;
    xstage_fwd_e<0, E>(v, cmk<C2>(1.0, 0.0));
    xstage_fwd_e<1, E>(v, tw[(N / 4) * (t & 1)]);
    xstage_fwd_e<2, E>(v, tw[(N / 8) * (t & 3)]);
#pragma unroll
    for (int k = 1; k < E; ++k) v[k] = cmul(v[k], tw[t * k]);
    if constexpr (PRUNE) dft4b_out_pruned<E / 4, -1>(v);
    else Dft<E, -1>::run(v);
}

// Line schedule of the z-plane kernel (defaults to FftCfg).  For 96 points
// 8 threads per line (12 work-group waves) with passes 4 x 6 x 4 measured
// fastest among 4 x 24 and 8 x 12 splits of the lines.
template <int N> struct PlaneCfg : FftCfg<N> {
    static constexpr int min_waves = 1;  // waves per SIMD the register budget must allow
};
template <> struct PlaneCfg<96> {
    static constexpr int N = 96, T = 8, E = 12, min_waves = 1;
    using Inv = RList<4, 6, 4>;
    using Fwd = RList<4, 6, 4>;
};
// Per precision (both precisions use the 96-point schedule above).  The
// FP32 plane (75 KB of LDS) caps its registers at 85 so that two
// work-groups share a compute unit: 0.147 against 0.158 ms per 53-band
// launch, despite a few spilled registers.
template <int N, class C2> struct PlaneCfgP : PlaneCfg<N> {};
template <> struct PlaneCfgP<96, float2> : PlaneCfg<96> {
    static constexpr int min_waves = 6;  // two 12-wave work-groups per compute unit
};

// Line schedules of the z-plane kernel that a plan can select (the
// autotuner times them on the plan's own shape).  Variant 0 is PlaneCfgP;
// the grids that run the Stockham passes (24 to 80 points) have two more,
// with other threads per line and radix orders.  Every list multiplies to
// N, each radix divides E = N / T, and the inverse list ends on the radix
// the forward list starts with, so the potential multiply stays in
// registers between them.
template <int N_, int T_, class Inv_, class Fwd_> struct SchedDef {
    static constexpr int N = N_, T = T_, E = N_ / T_, min_waves = 1;
    using Inv = Inv_;
    using Fwd = Fwd_;
};
template <int N, class C2, int V> struct PlaneSched : PlaneCfgP<N, C2> {};
template <class C2> struct PlaneSched<24, C2, 1> : SchedDef<24, 4, RList<6, 2, 2>, RList<2, 2, 6>> {};
template <class C2> struct PlaneSched<24, C2, 2> : SchedDef<24, 2, RList<4, 6>, RList<6, 4>> {};
template <class C2> struct PlaneSched<32, C2, 1> : SchedDef<32, 8, RList<4, 4, 2>, RList<2, 4, 4>> {};
template <class C2> struct PlaneSched<32, C2, 2> : SchedDef<32, 2, RList<16, 2>, RList<2, 16>> {};
template <class C2> struct PlaneSched<40, C2, 1> : SchedDef<40, 4, RList<10, 2, 2>, RList<2, 2, 10>> {};
template <class C2> struct PlaneSched<40, C2, 2> : SchedDef<40, 2, RList<20, 2>, RList<2, 20>> {};
template <class C2> struct PlaneSched<48, C2, 1> : SchedDef<48, 8, RList<6, 2, 2, 2>, RList<2, 2, 2, 6>> {};
template <class C2> struct PlaneSched<48, C2, 2> : SchedDef<48, 2, RList<12, 4>, RList<4, 12>> {};
template <class C2> struct PlaneSched<64, C2, 1> : SchedDef<64, 4, RList<16, 4>, RList<4, 16>> {};
template <class C2> struct PlaneSched<64, C2, 2> : SchedDef<64, 16, RList<4, 4, 4>, RList<4, 4, 4>> {};
template <class C2> struct PlaneSched<80, C2, 1> : SchedDef<80, 8, RList<10, 2, 2, 2>, RList<2, 2, 2, 10>> {};
template <class C2> struct PlaneSched<80, C2, 2> : SchedDef<80, 4, RList<4, 4, 5>, RList<5, 4, 4>> {};
// 96 points with four lanes per line, two threads of the cross-lane
// schedule in each (xlane96x2_inverse / xlane96x2_forward): 6 work-group
// waves, the potential in the same order as variant 0.  (The lists only
// satisfy the generic checks; the lines are cross-lane.)
template <class C2> struct PlaneSched<96, C2, 1> {
    static constexpr int N = 96, T = 4, E = 24, min_waves = sizeof(C2) == 8 ? 3 : 1;
    using Inv = RList<4, 6, 4>;
    using Fwd = RList<4, 6, 4>;
};
// 96 points, the compressed-column plane stage (plane_cc_body in apply.hip):
// the cross-lane lines of variant 0 and its potential order, the populated
// columns of one band at a time in LDS, two work-groups per compute unit
template <class C2> struct PlaneSched<96, C2, 2> : PlaneCfg<96> {
    static constexpr int min_waves = 4;  // two 8-wave work-groups per compute unit
};
// number of selectable schedules at N points
__host__ __device__ constexpr int plane_nsched(int n) { return n >= 24 && n <= 80 ? 3 : n == 96 ? 3 : 1; }
constexpr int kPlaneSchedMax = 3;

}  // namespace paro
