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

N, T, E = 96, 8, 12
PAIRS = {2: [(j, j + 6) for j in range(6)],
         1: [(j + 6 * c, j + 3 + 6 * c) for c in range(2) for j in range(3)],
         0: [(j, j + 6) for j in range(6)]}


def w(sign, m):
    return np.exp(sign * 2j * np.pi * m / N)


def stage_twiddle_exponent(b, t):
    return 12 * (t & 3) if b == 2 else (24 * (t & 1) if b == 1 else 0)


def xlane_index(t, s):
    return (s % 3 + 3 * (t >> 1 & 1) + 6 * (t >> 2 & 1)) + 12 * (4 * (s // 6) + 2 * (s // 3 % 2) + (t & 1))


def swap(R, b):
    """The lower lane (thread bit b clear) receives the upper lane's register s
    in s2; the upper lane receives the lower lane's s2 in s."""
    R = R.copy()
    for t in range(T):
        if t >> b & 1:
            continue
        u = t | (1 << b)
        for s, s2 in PAIRS[b]:
            R[t, s2], R[u, s] = R[u, s], R[t, s2]
    return R


def inverse(x):
    R = np.array([[x[t + T * m] for m in range(E)] for t in range(T)], dtype=complex)
    R = np.fft.ifft(R, axis=1) * E  # 12-point DFT with sign +1
    R = R * w(+1, np.outer(np.arange(T), np.arange(E)))
    for b in (2, 1, 0):
        R = swap(R, b)
        for t in range(T):
            tw = w(+1, stage_twiddle_exponent(b, t))
            for s, s2 in PAIRS[b]:
                u, v = R[t, s], R[t, s2]
                R[t, s], R[t, s2] = u + v, (u - v) * tw
    return R


def forward(R):
    R = R.copy()
    for b in (0, 1, 2):
        for t in range(T):
            twc = w(-1, stage_twiddle_exponent(b, t))
            for s, s2 in PAIRS[b]:
                a, c = R[t, s], R[t, s2] * twc
                R[t, s], R[t, s2] = a + c, a - c
        R = swap(R, b)
    R = R * w(-1, np.outer(np.arange(T), np.arange(E)))
    R = np.fft.fft(R, axis=1)  # 12-point DFT with sign -1
    out = np.empty(N, complex)
    for t in range(T):
        out[t + T * np.arange(E)] = R[t]
    return out


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
