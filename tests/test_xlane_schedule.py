"""The cross-lane 96-point schedule of the FP64 plane, stick and density
kernels, modelled lane by lane on the CPU: thread t of a line holds
x[t + 8 m]; a 12-point DFT in registers, the twiddle w^(t k1), then three
radix-2 decimation-in-frequency stages over the thread bits 2, 1, 0, each
after a swap of half the registers with the partner lane.  The model checks
that the register order the kernels assume (xlane_index in fft_device.h,
restated here) is where the DFT outputs land, that it is a bijection, and
that the forward transform (the conjugate transpose of every step, in
reverse) returns natural order.  No GPU and no oracle code involved: the
references are numpy's FFTs."""
import numpy as np
import pytest

T = 8


class Sched:
    """The schedule for N = 8 E points (E = 4 J registers: s = j + J d + 2 J e)."""

    def __init__(self, N):
        self.N, self.E = N, N // T
        J = self.J = self.E // 4
        self.pairs = {2: [(j, j + 2 * J) for j in range(2 * J)],
                      1: [(j + 2 * J * c, j + J + 2 * J * c) for c in range(2) for j in range(J)],
                      0: [(j, j + 2 * J) for j in range(2 * J)]}

    def w(self, sign, m):
        return np.exp(sign * 2j * np.pi * m / self.N)

    def stage_twiddle_exponent(self, b, t):
        return self.N // 8 * (t & 3) if b == 2 else (self.N // 4 * (t & 1) if b == 1 else 0)

    def xlane_index(self, t, s):
        J, E = self.J, self.E
        return (s % J + J * (t >> 1 & 1) + 2 * J * (t >> 2 & 1)) + E * (4 * (s // (2 * J)) + 2 * (s // J % 2) + (t & 1))

    def swap(self, R, b):
        """The lower lane (thread bit b clear) receives the upper lane's register s
        in s2; the upper lane receives the lower lane's s2 in s."""
        R = R.copy()
        for t in range(T):
            if t >> b & 1:
                continue
            u = t | (1 << b)
            for s, s2 in self.pairs[b]:
                R[t, s2], R[u, s] = R[u, s], R[t, s2]
        return R

    def inverse(self, x):
        E = self.E
        R = np.array([[x[t + T * m] for m in range(E)] for t in range(T)], dtype=complex)
        R = np.fft.ifft(R, axis=1) * E  # E-point DFT with sign +1
        R = R * self.w(+1, np.outer(np.arange(T), np.arange(E)))
        for b in (2, 1, 0):
            R = self.swap(R, b)
            for t in range(T):
                tw = self.w(+1, self.stage_twiddle_exponent(b, t))
                for s, s2 in self.pairs[b]:
                    u, v = R[t, s], R[t, s2]
                    R[t, s], R[t, s2] = u + v, (u - v) * tw
        return R

    def forward(self, R):
        E = self.E
        R = R.copy()
        for b in (0, 1, 2):
            for t in range(T):
                twc = self.w(-1, self.stage_twiddle_exponent(b, t))
                for s, s2 in self.pairs[b]:
                    a, c = R[t, s], R[t, s2] * twc
                    R[t, s], R[t, s2] = a + c, a - c
            R = self.swap(R, b)
        R = R * self.w(-1, np.outer(np.arange(T), np.arange(E)))
        R = np.fft.fft(R, axis=1)  # E-point DFT with sign -1
        out = np.empty(self.N, complex)
        for t in range(T):
            out[t + T * np.arange(E)] = R[t]
        return out


S96, S160 = Sched(96), Sched(160)
N, E = 96, 12


def xlane_index(t, s):
    return S96.xlane_index(t, s)


def inverse(x):
    return S96.inverse(x)


def forward(R):
    return S96.forward(R)


@pytest.mark.parametrize("n", [96, 160])
def test_register_order_is_a_bijection_both_lengths(n):
    S = Sched(n)
    assert sorted(S.xlane_index(t, s) for t in range(T) for s in range(S.E)) == list(range(n))
    if n == 96:  # the closed form the 96-point kernels use
        for t in range(T):
            for s in range(S.E):
                assert S.xlane_index(t, s) == (s % 3 + 3 * (t >> 1 & 1) + 6 * (t >> 2 & 1)) + 12 * (
                    4 * (s // 6) + 2 * (s // 3 % 2) + (t & 1))


@pytest.mark.parametrize("seed", [0, 1])
def test_160_point_schedule_inverse_and_convolution_step(seed):
    """The same four-step schedule with a 20-point DFT in registers (160 = 20 x 8)."""
    S = S160
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(160) + 1j * rng.standard_normal(160)
    X = np.fft.ifft(x) * 160
    R = S.inverse(x)
    assert max(abs(R[t, s] - X[S.xlane_index(t, s)]) for t in range(T) for s in range(S.E)) < 1e-12 * np.abs(X).max()
    V = rng.standard_normal(160)
    Vr = np.array([[V[S.xlane_index(t, s)] for s in range(S.E)] for t in range(T)])
    y = S.forward(R * Vr)
    ref = np.fft.fft(V * X)
    assert np.abs(y - ref).max() < 1e-11 * np.abs(ref).max()


def test_register_order_is_a_bijection():
    assert sorted(xlane_index(t, s) for t in range(T) for s in range(E)) == list(range(N))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_inverse_lands_in_register_order(seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    X = np.fft.ifft(x) * N  # unnormalised, sign +1
    R = inverse(x)
    got = np.array([[R[t, s] - X[xlane_index(t, s)] for s in range(E)] for t in range(T)])
    assert np.abs(got).max() < 1e-12 * np.abs(X).max()


@pytest.mark.parametrize("seed", [3, 4])
def test_forward_of_multiplied_block_is_the_convolution_step(seed):
    """forward(V * inverse(x)) in register order = FFT(V * IFFT(x)) in natural order,
    the potential step of the plane stage with V laid out by xlane_index."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    V = rng.standard_normal(N)
    R = inverse(x)
    Vr = np.array([[V[xlane_index(t, s)] for s in range(E)] for t in range(T)])
    y = forward(R * Vr)
    ref = np.fft.fft(V * (np.fft.ifft(x) * N))
    assert np.abs(y - ref).max() < 1e-11 * np.abs(ref).max()


def test_pruned_positions_are_never_populated_on_accepted_grids():
    """Plans need N >= 4 n_max + 1, so at N = 96 every n_max <= 23, and no
    populated index i = n mod 96 (|n| <= n_max) sits at a pruned position
    t + 8 m with m = 3..8 (the kernels neither load nor store those)."""
    nmax_limit = max(n for n in range(96) if 96 >= 4 * n + 1)
    assert nmax_limit == 23
    for nmax in range(nmax_limit + 1):
        for n in range(-nmax, nmax + 1):
            i = n % N
            assert not 3 <= i // T <= 8, (nmax, n)
    # and a line with only those positions populated transforms like the full one
    rng = np.random.default_rng(5)
    x = np.zeros(N, complex)
    kept = [i for i in range(N) if not 3 <= i // T <= 8]
    x[kept] = rng.standard_normal(len(kept)) + 1j * rng.standard_normal(len(kept))
    R = inverse(x)
    X = np.fft.ifft(x) * N
    assert max(abs(R[t, s] - X[xlane_index(t, s)]) for t in range(T) for s in range(E)) < 1e-12 * np.abs(X).max()


# ---------------------------------------------------------------- pruned 12-point DFTs
# The 96-point kernels take the 12-point DFT in registers as 12 = 4 x 3:
# input m = s_b + 3 q (q < 4), a 4-point DFT over q, the twiddle
# w12^(s_b k_a), a 3-point DFT over s_b, output k = k_a + 4 k_b.  With
# inputs 3..8 zero (q = 1, 2) the 4-point DFTs see only q = 0 and 3
# (dft12_in_pruned); of the outputs only k = 0, 1, 2, 9, 10, 11 are kept
# (k_b = 0 for k_a < 3, k_b = 2 for k_a > 0: dft12_out_pruned).  The model
# restates those two steps and checks them against numpy.

def _dft(x, sign):
    n = len(x)
    k = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(k, k) / n) @ x


def dft12_in_pruned_model(v, sign):
    y = np.zeros(12, complex)
    for sb in range(3):
        a0, a3 = v[sb], v[9 + sb]
        d = sign * 1j * a3
        y[sb * 4 + 0], y[sb * 4 + 2] = a0 + a3, a0 - a3
        y[sb * 4 + 1], y[sb * 4 + 3] = a0 - d, a0 + d
    out = np.zeros(12, complex)
    for ka in range(4):
        b = np.array([y[ka], y[4 + ka], y[8 + ka]]) * np.exp(sign * 2j * np.pi * np.arange(3) * ka / 12)
        out[ka + 4 * np.arange(3)] = _dft(b, sign)
    return out


def dft12_out_pruned_model(v, sign):
    y = np.zeros(12, complex)
    for sb in range(3):
        y[sb * 4:sb * 4 + 4] = _dft(np.array([v[sb], v[3 + sb], v[6 + sb], v[9 + sb]]), sign)
    out = np.full(12, np.nan + 0j)
    h = np.sin(2 * np.pi / 3)
    for ka in range(4):
        b = np.array([y[ka], y[4 + ka], y[8 + ka]]) * np.exp(sign * 2j * np.pi * np.arange(3) * ka / 12)
        t1 = b[1] + b[2]
        if ka < 3:
            out[ka] = b[0] + t1
        if ka > 0:
            out[ka + 8] = (b[0] - 0.5 * t1) - sign * 1j * h * (b[1] - b[2])
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pruned_dft12_inverse_on_zero_inputs(seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    v[3:9] = 0.0
    assert np.abs(dft12_in_pruned_model(v, +1) - np.fft.ifft(v) * 12).max() < 1e-13
    # the pruning really assumes those inputs zero: a nonzero one is dropped
    w = v.copy()
    w[5] = 1.0
    assert np.abs(dft12_in_pruned_model(w, +1) - np.fft.ifft(w) * 12).max() > 0.1


@pytest.mark.parametrize("seed", [3, 4])
def test_pruned_dft12_forward_kept_outputs(seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    got = dft12_out_pruned_model(v, -1)
    kept = [0, 1, 2, 9, 10, 11]
    assert np.abs(got[kept] - np.fft.fft(v)[kept]).max() < 1e-13
    assert np.all(np.isnan(got[3:9]))
    assert [m for m in range(12) if not 3 <= m <= 8] == kept


# The same pruning for the 160-point lines (E = 20 = 4 x 5, dft4b_in_pruned /
# dft4b_out_pruned with B = 5): every populated |n| <= 39, so x[t + 8 m] is
# zero for m = 5..14 (s_a = 1, 2 of the 4-point DFTs over x[5 s_a + s_b]) and
# only the outputs m < 5 or m >= 15 are kept.  The model restates the
# generic steps for B = 3 and 5 and checks them against numpy.

def kept_e(E, m):
    return m < E // 4 or m >= 3 * E // 4


def dft4b_in_pruned_model(v, sign, B):
    E = 4 * B
    y = np.zeros(E, complex)
    for sb in range(B):
        a0, a3 = v[sb], v[3 * B + sb]
        d = sign * 1j * a3
        y[sb * 4 + 0], y[sb * 4 + 2] = a0 + a3, a0 - a3
        y[sb * 4 + 1], y[sb * 4 + 3] = a0 - d, a0 + d
    out = np.zeros(E, complex)
    for ka in range(4):
        b = np.array([y[sb * 4 + ka] for sb in range(B)]) * np.exp(sign * 2j * np.pi * np.arange(B) * ka / E)
        out[ka + 4 * np.arange(B)] = _dft(b, sign)
    return out


def dft4b_out_pruned_model(v, sign, B):
    E = 4 * B
    y = np.zeros(E, complex)
    for sb in range(B):
        y[sb * 4:sb * 4 + 4] = _dft(np.array([v[sb], v[B + sb], v[2 * B + sb], v[3 * B + sb]]), sign)
    out = np.full(E, np.nan + 0j)
    for ka in range(4):
        b = np.array([y[sb * 4 + ka] for sb in range(B)]) * np.exp(sign * 2j * np.pi * np.arange(B) * ka / E)
        full = _dft(b, sign)
        for kb in range(B):
            if kept_e(E, ka + 4 * kb):
                out[ka + 4 * kb] = full[kb]
    return out


@pytest.mark.parametrize("B,seed", [(3, 5), (5, 6), (5, 7)])
def test_pruned_dft4b_inverse_on_zero_inputs(B, seed):
    E = 4 * B
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(E) + 1j * rng.standard_normal(E)
    v[B:3 * B] = 0.0
    assert np.abs(dft4b_in_pruned_model(v, +1, B) - np.fft.ifft(v) * E).max() < 1e-13
    if B == 3:
        assert np.abs(dft4b_in_pruned_model(v, +1, B) - dft12_in_pruned_model(v, +1)).max() < 1e-14
    w = v.copy()
    w[B + 1] = 1.0
    assert np.abs(dft4b_in_pruned_model(w, +1, B) - np.fft.ifft(w) * E).max() > 0.1


@pytest.mark.parametrize("B,seed", [(3, 8), (5, 9)])
def test_pruned_dft4b_forward_kept_outputs(B, seed):
    E = 4 * B
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(E) + 1j * rng.standard_normal(E)
    got = dft4b_out_pruned_model(v, -1, B)
    kept = [m for m in range(E) if kept_e(E, m)]
    assert len(kept) == E // 2
    assert np.abs(got[kept] - np.fft.fft(v)[kept]).max() < 1e-13
    assert np.all(np.isnan(np.delete(got, kept)))


def test_pruned_160_positions_cover_every_populated_index():
    """x[t + 8 m] of a 160-point line with m kept covers every |n| <= 39, the
    largest n_max a 160-point plan accepts (160 >= 4 n_max + 1)."""
    nmax = (160 - 1) // 4
    assert nmax == 39
    for t in range(8):
        for m in range(20):
            i = t + 8 * m
            n = i if i < 80 else i - 160
            if abs(n) <= nmax:
                assert kept_e(20, m), (t, m)


# ---------------------------------------------------------------- two threads per lane
# Plane schedule 1 at 96 points runs the same schedule with threads 2 u
# (set a) and 2 u + 1 (set b) in one lane: the stages on thread bits 2 and 1
# are the swaps above, once per set; the stage on thread bit 0 becomes a
# renaming of registers inside the lane (xstage_inv_bit0 / xstage_fwd_bit0
# in fft_device.h, restated here).

def pair_bit0_inverse(a, b):
    a2, b2 = a.copy(), b.copy()
    for i in range(6):
        pa, qa, pb, qb = a[i], b[i], a[i + 6], b[i + 6]
        a2[i], a2[i + 6] = pa + qa, pa - qa
        b2[i], b2[i + 6] = pb + qb, pb - qb
    return a2, b2


def pair_bit0_forward(a, b):
    a2, b2 = a.copy(), b.copy()
    for i in range(6):
        a2[i], a2[i + 6] = a[i] + a[i + 6], b[i] + b[i + 6]
        b2[i], b2[i + 6] = a[i] - a[i + 6], b[i] - b[i + 6]
    return a2, b2


def _bit0_stage_inverse(R):
    R = S96.swap(R, 0)
    for t in range(T):
        for s, s2 in S96.pairs[0]:
            u, v = R[t, s], R[t, s2]
            R[t, s], R[t, s2] = u + v, u - v
    return R


def _bit0_stage_forward(R):
    R = R.copy()
    for t in range(T):
        for s, s2 in S96.pairs[0]:
            a, c = R[t, s], R[t, s2]
            R[t, s], R[t, s2] = a + c, a - c
    return S96.swap(R, 0)


@pytest.mark.parametrize("seed", [0, 1])
def test_paired_bit0_stage_is_the_swap_stage(seed):
    """On any register state the in-lane stage of each direction gives lane u's
    sets exactly the registers threads 2 u and 2 u + 1 hold after the
    eight-lane swap stage."""
    rng = np.random.default_rng(seed)
    R = rng.standard_normal((T, E)) + 1j * rng.standard_normal((T, E))
    for stage8, stage2 in ((_bit0_stage_inverse, pair_bit0_inverse), (_bit0_stage_forward, pair_bit0_forward)):
        ref = stage8(R)
        for u in range(4):
            a, b = stage2(R[2 * u], R[2 * u + 1])
            assert np.array_equal(a, ref[2 * u]) and np.array_equal(b, ref[2 * u + 1])


@pytest.mark.parametrize("seed", [5, 6])
def test_paired_schedule_convolution_step(seed):
    """The whole paired row step, inverse, x V in the lane's 24-value order
    (set a then set b), forward, against numpy."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    V = rng.standard_normal(N)
    # inverse: per-thread DFT, twiddle and the bit-2 and bit-1 stages, then the in-lane bit-0 stage
    R = np.array([[x[t + T * m] for m in range(E)] for t in range(T)], dtype=complex)
    R = np.fft.ifft(R, axis=1) * E
    R = R * S96.w(+1, np.outer(np.arange(T), np.arange(E)))
    for b in (2, 1):
        R = S96.swap(R, b)
        for t in range(T):
            tw = S96.w(+1, S96.stage_twiddle_exponent(b, t))
            for s, s2 in S96.pairs[b]:
                u, v = R[t, s], R[t, s2]
                R[t, s], R[t, s2] = u + v, (u - v) * tw
    lanes = [pair_bit0_inverse(R[2 * u], R[2 * u + 1]) for u in range(4)]
    X = np.fft.ifft(x) * N
    for u, (a, b) in enumerate(lanes):
        for s in range(E):
            assert abs(a[s] - X[xlane_index(2 * u, s)]) < 1e-12 * np.abs(X).max()
            assert abs(b[s] - X[xlane_index(2 * u + 1, s)]) < 1e-12 * np.abs(X).max()
    # lane u's potential: 24 values, position p = 24 u + e of the row (the same
    # memory order as eight threads of 12)
    Vl = np.array([V[xlane_index(2 * u + e // 12, e % 12)] for u in range(4) for e in range(24)]).reshape(4, 24)
    lanes = [(a * Vl[u, :12], b * Vl[u, 12:]) for u, (a, b) in enumerate(lanes)]
    # forward: in-lane bit-0 stage, then the eight-lane bit-1 and bit-2 stages and the rest
    R = np.zeros((T, E), complex)
    for u, (a, b) in enumerate(lanes):
        R[2 * u], R[2 * u + 1] = pair_bit0_forward(a, b)
    for b in (1, 2):
        for t in range(T):
            twc = S96.w(-1, S96.stage_twiddle_exponent(b, t))
            for s, s2 in S96.pairs[b]:
                a_, c = R[t, s], R[t, s2] * twc
                R[t, s], R[t, s2] = a_ + c, a_ - c
        R = S96.swap(R, b)
    R = R * S96.w(-1, np.outer(np.arange(T), np.arange(E)))
    R = np.fft.fft(R, axis=1)
    y = np.empty(N, complex)
    for t in range(T):
        y[t + T * np.arange(E)] = R[t]
    ref = np.fft.fft(V * X)
    assert np.abs(y - ref).max() < 1e-11 * np.abs(ref).max()
