"""CPU model of the plane kernel's Stockham line schedules, every selectable one.

The schedules are read from the kernel header (FftCfg for schedule 0,
PlaneSched specialisations for the others), so the model runs exactly the
configurations the library compiles.  Thread t of a line holds E = N / T
values; a radix-R pass at stride NS loads v[q R + r] = x[t + T q + r N/R],
twiddles by w^(r k N / (NS R)) with k = (t + T q) mod NS, runs R-point DFTs
and stores to (j // NS) NS R + j mod NS + r NS.  After the last pass (radix
RL) v[q RL + r] is element t + T q + r N / RL: that is the order the plane
potential is laid out in, and the forward list must start with RL so that
the multiply needs no exchange.
"""
import os
import re

import numpy as np
import pytest

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_1702_04045_amd", "csrc", "fft_device.h")


def _rlist(s):
    return [int(v) for v in s.replace(" ", "").split(",")]


def schedules():
    src = open(HDR).read()
    out = {}
    for m in re.finditer(r"struct FftCfg<(\d+)> \{ static constexpr int N = \d+, T = (\d+), E = (\d+); "
                         r"using Inv = RList<([\d, ]+)>; using Fwd = RList<([\d, ]+)>; \};", src):
        n = int(m.group(1))
        out[(n, 0)] = (int(m.group(2)), _rlist(m.group(4)), _rlist(m.group(5)))
    for m in re.finditer(r"struct PlaneSched<(\d+), C2, (\d+)> : SchedDef<(\d+), (\d+), RList<([\d, ]+)>, "
                         r"RList<([\d, ]+)>>", src):
        n, v = int(m.group(1)), int(m.group(2))
        assert int(m.group(3)) == n
        out[(n, v)] = (int(m.group(4)), _rlist(m.group(5)), _rlist(m.group(6)))
    return out


SCHED = schedules()
STOCKHAM = sorted(k for k in SCHED if 24 <= k[0] <= 80)


def test_header_has_three_schedules_per_stockham_grid():
    for n in (24, 32, 40, 48, 64, 80):
        assert [(n, v) in SCHED for v in range(3)] == [True] * 3, n
    assert len(STOCKHAM) == 18


def dft(v, sign):
    R = len(v)
    k = np.arange(R)
    return np.exp(sign * 2j * np.pi * np.outer(k, k) / R) @ v


def run_line(x_or_regs, N, T, rlist, sign, loaded=False):
    """Model of the stockham passes of one line; returns registers v[t][e]."""
    E = N // T
    line = np.zeros(N, complex)
    R0 = rlist[0]
    if loaded:
        v = [np.array(r, complex) for r in x_or_regs]
    else:
        x = x_or_regs
        v = [np.array([x[t + T * q + r * (N // R0)] for q in range(E // R0) for r in range(R0)]) for t in range(T)]
    NS = 1
    for i, R in enumerate(rlist):
        for t in range(T):
            for q in range(E // R):
                blk = v[t][q * R:(q + 1) * R].copy()
                if NS > 1:
                    k = (t + T * q) % NS
                    for r in range(1, R):
                        blk[r] *= np.exp(sign * 2j * np.pi * (r * k * (N // (NS * R))) / N)
                v[t][q * R:(q + 1) * R] = dft(blk, sign)
        if i + 1 < len(rlist):
            for t in range(T):
                for q in range(E // R):
                    j = t + T * q
                    base = (j // NS) * NS * R + j % NS
                    for r in range(R):
                        line[base + r * NS] = v[t][q * R + r]
            R2 = rlist[i + 1]
            for t in range(T):
                v[t] = np.array([line[t + T * q + r * (N // R2)] for q in range(E // R2) for r in range(R2)])
            NS *= R
    return v


def final_index(N, T, RL, t, e):
    return t + T * (e // RL) + (e % RL) * (N // RL)


@pytest.mark.parametrize("key", STOCKHAM, ids=[f"n{n}_s{v}" for n, v in STOCKHAM])
def test_schedule_constraints(key):
    N, _ = key
    T, inv, fwd = SCHED[key]
    E = N // T
    assert T * E == N and 64 % T == 0 and N * T <= 1024
    for lst in (inv, fwd):
        assert int(np.prod(lst)) == N
        assert all(E % R == 0 for R in lst)
    assert inv[-1] == fwd[0]
    # the potential order is a bijection onto the row
    idx = sorted(final_index(N, T, inv[-1], t, e) for t in range(T) for e in range(E))
    assert idx == list(range(N))


@pytest.mark.parametrize("key", STOCKHAM, ids=[f"n{n}_s{v}" for n, v in STOCKHAM])
def test_inverse_and_forward_are_dfts(key):
    N, _ = key
    T, inv, fwd = SCHED[key]
    E = N // T
    rng = np.random.default_rng(N)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    for sign, lst in ((+1, inv), (-1, fwd)):
        v = run_line(x, N, T, lst, sign)
        got = np.zeros(N, complex)
        for t in range(T):
            for e in range(E):
                got[final_index(N, T, lst[-1], t, e)] = v[t][e]
        ref = np.fft.ifft(x) * N if sign > 0 else np.fft.fft(x)
        assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("key", STOCKHAM, ids=[f"n{n}_s{v}" for n, v in STOCKHAM])
def test_row_step_multiplies_in_registers(key):
    """Inverse, multiply by the potential in the layout order, forward from the
    same registers: the row of the plane stage (convolution with V)."""
    N, _ = key
    T, inv, fwd = SCHED[key]
    E = N // T
    rng = np.random.default_rng(N + 1)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    V = rng.standard_normal(N)
    v = run_line(x, N, T, inv, +1)
    for t in range(T):
        for e in range(E):
            v[t][e] *= V[final_index(N, T, inv[-1], t, e)]
    w = run_line(v, N, T, fwd, -1, loaded=True)
    got = np.zeros(N, complex)
    for t in range(T):
        for e in range(E):
            got[final_index(N, T, fwd[-1], t, e)] = w[t][e]
    ref = np.fft.fft(V * (np.fft.ifft(x) * N))
    assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max()
