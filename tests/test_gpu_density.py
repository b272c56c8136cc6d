"""GPU density (paro_density) and projector gradient (paro_projector_gradient)
against the oracle, and the Hellmann-Feynman gradients of the band energy
against central finite differences of the device eigensolver.

Tolerances:
  density                      max |diff| <= 1e-12 max |ref| (two FP64 FFT stages
                               and a square; sums in a fixed band order)
  projector gradient           max |diff| <= 1e-12 max |ref| (FP64 products of
                               length n_g; the oracle sums directly)
  gradient vs finite diff.     |g.d - FD| <= 1e-6 max(|FD|, |g| |d|): the
                               Hellmann-Feynman error is first order in the
                               eigenvector error (residual 1e-10 over a gap of
                               ~0.01 Ha); the central difference with h = 1e-4 has
                               O(h^2) truncation and 1e-14 / h rounding
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def make_case(spec, seed=0):
    import paper_1702_04045_amd as P
    c = synth.make_cell(spec, seed)
    v = synth.vloc_on_grid(c["cell"], c["grid"], c["positions"], c["depths"], c["widths"])
    h = oracle.Hamiltonian(c["cell"], c["ecut"], v, c["projectors"])
    pl = P.Plan(c["cell"], c["ecut"], v, c["projectors"])
    assert pl.ng == h.ng
    return c, v, h, pl


def to_dev(x):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def to_np(t):
    return t.detach().cpu().numpy()


def rel_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


TINY = synth.small_cell(a=6.0, ecut=4.0, grid=16, n_atoms=2)
C0 = synth.WORKLOADS["c0"]
C1 = synth.WORKLOADS["c1"]


@pytest.mark.parametrize("spec,nb,weighted", [(TINY, 3, False), (C0, 8, True), (C0, 13, True), (C0, 1, False),
                                              (C0, 70, True)],
                         ids=["tiny", "c0_8", "c0_odd13", "c0_1", "c0_two_chunks70"])
def test_density_matches_oracle(spec, nb, weighted):
    c, v, h, pl = make_case(spec, 4)
    x = synth.trial_block(h.ng, nb, 4)
    w = np.linspace(2.0, 0.25, nb) if weighted else None
    ref = h.density(x, w)
    got = to_np(pl.density(to_dev(x), None if w is None else to_dev(w)))
    assert got.shape == ref.shape
    assert rel_err(got, ref) < 1e-12


@pytest.mark.parametrize("grid", [8, 24, 32, 40, 48, 64, 80, 96])
def test_density_every_supported_grid(grid):
    """Every instantiated plane length: two bands per column stage up to 64
    points, one band per stage with LDS-held sums at 80 and 96."""
    spec = synth.small_cell(a=4.0, ecut=2.5, grid=grid, n_atoms=2) if grid == 8 else \
        synth.small_cell(a=6.0, ecut=4.0, grid=grid, n_atoms=2)
    c, v, h, pl = make_case(spec, 5)
    for nb in (1, 5, 9):
        x = synth.trial_block(h.ng, nb, nb)
        w = np.linspace(1.0, 3.0, nb)
        assert rel_err(to_np(pl.density(to_dev(x), to_dev(w))), h.density(x, w)) < 1e-12, nb


def test_density_padded_leading_dimension_and_repeatability():
    torch = _torch()
    c, v, h, pl = make_case(C0, 6)
    x = synth.trial_block(h.ng, 11, 6)
    xd = torch.zeros((11, h.ng + 21), dtype=torch.complex128, device="cuda:0")
    xd[:, :h.ng] = to_dev(x)
    xd[:, h.ng:] = 1e3  # padding must not be read
    a = pl.density(xd)
    b = pl.density(xd)
    assert (a == b).all().item()
    assert rel_err(to_np(a), h.density(x)) < 1e-12


def test_density_full_size_sampled_bands():
    """The 96^3 grid of the 34k-plane-wave cell, all 160 bands in one call (the
    solver's block size, three 64-band chunks); weights zero except on four
    bands, which the oracle sums directly."""
    c, v, h, pl = make_case(C1, 0)
    nb = C1.n_carried
    x = synth.trial_block(h.ng, nb, 0)
    w = np.zeros(nb)
    idx = [0, 63, 64, nb - 1]
    w[idx] = [1.0, 0.5, 2.0, 1.5]
    got = to_np(pl.density(to_dev(x), to_dev(w)))
    ref = h.density(x[idx], w[idx])
    assert rel_err(got, ref) < 1e-12
    # all bands, unit weights: Parseval, sum_j rho_j = N sum_b ||c_b||^2
    tot = to_np(pl.density(to_dev(x))).sum()
    assert abs(tot - np.prod(h.grid) * (np.abs(x) ** 2).sum()) < 1e-11 * tot


def test_density_argument_errors():
    import ctypes as C

    import paper_1702_04045_amd as P
    torch = _torch()
    c, v, h, pl = make_case(TINY, 0)
    x = to_dev(synth.trial_block(h.ng, 2, 0))
    rho = torch.empty(pl.grid, dtype=torch.float64, device="cuda:0")
    n = C.c_size_t()
    assert pl.lib.paro_density_workspace_bytes(pl.h, 2, C.byref(n)) == 0
    ws = torch.empty(n.value + 256, dtype=torch.uint8, device="cuda:0")
    base = ws.data_ptr() + (-ws.data_ptr()) % 256
    vp = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
    assert pl.lib.paro_density(pl.h, 0, vp(x), h.ng, None, vp(rho), C.c_void_p(base), n.value) == P._lib.PARO_EINVAL
    assert pl.lib.paro_density(pl.h, 2, vp(x), h.ng - 1, None, vp(rho), C.c_void_p(base), n.value) == P._lib.PARO_EINVAL
    assert pl.lib.paro_density(pl.h, 2, vp(x), h.ng, None, vp(rho), C.c_void_p(base), n.value - 1) == P._lib.PARO_ESIZE
    assert pl.lib.paro_density(pl.h, 2, vp(x), h.ng, None, vp(rho), C.c_void_p(base + 8), n.value) == P._lib.PARO_EINVAL
    assert pl.lib.paro_density(pl.h, 2, vp(x), h.ng, None, vp(rho), C.c_void_p(base), n.value) == 0
    torch.cuda.synchronize()


# ---------------------------------------------------------------- band-energy gradient

def _problem(spec, seed, n_occ, tol=1e-10):
    from paper_1702_04045_amd.grad import BandEnergyProblem
    c = synth.make_cell(spec, seed)
    v = synth.vloc_on_grid(c["cell"], c["grid"], c["positions"], c["depths"], c["widths"])
    ng = len(oracle.sphere(c["cell"], c["ecut"])[0])
    n_bands = n_occ + 4
    prob = BandEnergyProblem(c["cell"], c["ecut"], c["projectors"], n_occ, n_bands=n_bands,
                             weights=np.linspace(2.0, 1.0, n_occ), trial=synth.trial_block(ng, n_bands, seed),
                             tol_res=tol)
    return c, v, prob


def test_band_energy_gradient_is_the_oracle_density():
    """Backward of the band energy equals the oracle's density of the converged
    block over N, and the energy equals the dense eigenvalue sum."""
    torch = _torch()
    from paper_1702_04045_amd.grad import band_energy
    c, v, prob = _problem(C0, 0, 6)
    V = torch.tensor(v, dtype=torch.float64, requires_grad=True)
    E = band_energy(V, prob)
    E.backward()
    h = oracle.Hamiltonian(c["cell"], c["ecut"], v, c["projectors"])
    lam = np.linalg.eigvalsh(h.dense())
    w = np.linspace(2.0, 1.0, 6)
    assert abs(E.item() - w @ lam[:6]) < 1e-10 * abs(w @ lam[:6])
    psi = to_np(prob.last[0])[:6, :h.ng]
    ref = h.density(psi, w) / np.prod(h.grid)
    assert V.grad.shape == v.shape
    assert rel_err(V.grad.numpy(), ref) < 1e-11


def test_band_energy_gradient_matches_finite_differences():
    """Directional derivatives along 20 random smooth directions: the
    Hellmann-Feynman gradient against central differences of the converged
    device eigenvalue sum."""
    torch = _torch()
    from paper_1702_04045_amd.grad import band_energy
    c, v, prob = _problem(C0, 1, 6)
    V = torch.tensor(v, dtype=torch.float64, requires_grad=True)
    E = band_energy(V, prob)
    (g,) = torch.autograd.grad(E, V)
    g = g.numpy()
    rng = np.random.default_rng(20)
    hstep = 1e-4
    grid = np.array(v.shape)
    J = np.indices(v.shape).reshape(3, -1).T / grid
    for k in range(20):
        # a few random Fourier modes with random phases, unit max norm
        d = np.zeros(v.size)
        for _ in range(3):
            n = rng.integers(-4, 5, size=3)
            d += rng.standard_normal() * np.cos(2 * np.pi * (J @ n) + rng.uniform(0, 2 * np.pi))
        d = (d / np.abs(d).max()).reshape(v.shape)
        ep = band_energy(torch.tensor(v + hstep * d), prob).item()
        em = band_energy(torch.tensor(v - hstep * d), prob).item()
        fd = (ep - em) / (2 * hstep)
        an = float((g * d).sum())
        assert abs(an - fd) <= 1e-6 * max(abs(fd), np.abs(g).sum()), (k, an, fd)


# ---------------------------------------------------------------- projector gradient

MED = synth.small_cell(a=8.0, ecut=6.0, grid=24, n_atoms=3)


@pytest.mark.parametrize("spec,nb,weighted", [(TINY, 3, False), (MED, 9, True), (MED, 1, True)],
                         ids=["tiny", "med9", "med1"])
def test_projector_gradient_matches_oracle(spec, nb, weighted):
    c, v, h, pl = make_case(spec, 7)
    x = synth.trial_block(h.ng, nb, 7)
    w = np.linspace(0.5, 2.0, nb) if weighted else None
    dd_ref, dR_ref = h.projector_gradient(x, w)
    dd, dR = pl.projector_gradient(to_dev(x), None if w is None else to_dev(w))
    assert rel_err(to_np(dd), dd_ref) < 1e-12
    assert rel_err(to_np(dR), dR_ref) < 1e-12


def test_projector_gradient_full_size_sampled_bands():
    """128 projectors, all 160 bands of the benchmark cell in one call;
    weights zero except on four bands, which the oracle sums directly."""
    c, v, h, pl = make_case(C1, 0)
    nb = C1.n_carried
    x = synth.trial_block(h.ng, nb, 1)
    w = np.zeros(nb)
    idx = [0, 63, 64, nb - 1]
    w[idx] = [1.0, 0.5, 2.0, 1.5]
    dd, dR = pl.projector_gradient(to_dev(x), to_dev(w))
    dd_ref, dR_ref = h.projector_gradient(x[idx], w[idx])
    assert rel_err(to_np(dd), dd_ref) < 1e-12
    assert rel_err(to_np(dR), dR_ref) < 1e-12
    dd2, dR2 = pl.projector_gradient(to_dev(x), to_dev(w))
    assert (dd2 == dd).all().item() and (dR2 == dR).all().item()


def test_band_energy_projector_gradients_match_finite_differences():
    """d E / d R_p and d E / d d_p from the backward pass against
    Richardson-extrapolated central differences of the converged device
    eigenvalue sum, on a cell with 12 projectors."""
    torch = _torch()
    from paper_1702_04045_amd.grad import band_energy
    c, v, prob = _problem(MED, 3, 4)
    V = torch.tensor(v, dtype=torch.float64)
    R = torch.tensor([list(p["center"]) for p in c["projectors"]], dtype=torch.float64, requires_grad=True)
    D = torch.tensor([p["d"] for p in c["projectors"]], dtype=torch.float64, requires_grad=True)
    E = band_energy(V, prob, R, D)
    gR, gD = torch.autograd.grad(E, (R, D))
    gR, gD = gR.numpy(), gD.numpy()
    scale = max(np.abs(gR).max(), np.abs(gD).max())

    def energy(Rm, Dm):
        return band_energy(V, prob, torch.tensor(Rm), torch.tensor(Dm)).item()

    def deriv(f, h=1e-4):
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        return (4 * d2 - d1) / 3

    R0, D0 = R.detach().numpy(), D.detach().numpy()
    for p in (0, 1, 5, 11):
        def fd_d(s, p=p):
            Dm = D0.copy()
            Dm[p] += s
            return energy(R0, Dm)
        assert abs(deriv(fd_d) - gD[p]) <= 1e-6 * scale, ("d", p)
        for a in range(3):
            def fd_r(s, p=p, a=a):
                Rm = R0.copy()
                Rm[p, a] += s
                return energy(Rm, D0)
            assert abs(deriv(fd_r) - gR[p, a]) <= 1e-6 * scale, ("R", p, a)
