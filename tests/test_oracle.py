"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: brute-force
enumeration, a library routine (numpy's FFT, LAPACK eigh/solve/cholesky),
a closed form (free electrons, constant and cosine potentials, the rank-one
secular equation) or an invariant (Hermiticity, translation invariance,
Courant-Fischer, the fixed point of the ParO map).  A plausible mistake in
the oracle (a wrong sign of the FFT or projector phase, a dropped kinetic or
nonlocal term, a transposed Gram matrix) fails at least one of them.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def brute_sphere(cell, ecut):
    b = 2 * np.pi * np.linalg.inv(np.asarray(cell, float)).T
    gmax = np.sqrt(2 * ecut)
    out = []
    # a generous box: |n_d| <= gmax |a_d| / 2pi + 2
    box = [int(gmax * np.linalg.norm(cell[d]) / (2 * np.pi)) + 2 for d in range(3)]
    for n in itertools.product(*[range(-m, m + 1) for m in box]):
        G = np.array(n) @ b
        if 0.5 * G @ G <= ecut * (1 + 1e-12):
            out.append(n)
    return np.array(out, np.int32)


def cell_data(spec, seed=0):
    c = synth.make_cell(spec, seed)
    v = synth.vloc_on_grid(c["cell"], c["grid"], c["positions"], c["depths"], c["widths"])
    return c, v


def tiny(seed=0, **kw):
    spec = synth.small_cell(**kw)
    c, v = cell_data(spec, seed)
    return spec, c, v, oracle.Hamiltonian(c["cell"], c["ecut"], v, c["projectors"])


# ---------------------------------------------------------------- sphere (e3)

@pytest.mark.parametrize("cell,ecut", [
    (np.eye(3) * 6.0, 4.0),
    (np.diag([5.0, 6.5, 7.0]), 5.0),
    (np.array([[5.0, 0, 0], [1.2, 5.5, 0], [0.3, -0.7, 6.0]]), 3.5),
    (np.eye(3) * 10.0, 10.0),
])
def test_sphere_matches_brute_force(cell, ecut):
    mil, nmax = oracle.sphere(cell, ecut)
    ref = brute_sphere(cell, ecut)
    # lexicographic order == itertools.product order of the brute force
    assert np.array_equal(mil, ref)
    assert np.array_equal(nmax, np.abs(ref).max(axis=0))


def test_sphere_counts_of_the_workloads():
    # counts for the 10 Ha / 10 bohr and 20 Ha / 20 bohr cubic cells, checked
    # against brute force for the first and against the free-electron volume
    # estimate Omega (2 E_cut)^(3/2) / (6 pi^2) for both
    for key, brute in (("c0", True), ("c1", False)):
        s = synth.WORKLOADS[key]
        mil, nmax = oracle.sphere(s.cell, s.ecut)
        if brute:
            assert len(mil) == len(brute_sphere(s.cell, s.ecut))
        est = s.a ** 3 * (2 * s.ecut) ** 1.5 / (6 * np.pi ** 2)
        assert abs(len(mil) - est) / est < 0.01
        assert s.grid >= 4 * nmax.max() + 1
    assert len(oracle.sphere(synth.WORKLOADS["c0"].cell, 10.0)[0]) == 1503
    assert len(oracle.sphere(synth.WORKLOADS["c1"].cell, 20.0)[0]) == 34265


# ---------------------------------------------------------------- FFT

@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft1d_vs_dft_definition(n, sign):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    j = np.arange(n)
    F = np.exp(sign * 2j * np.pi * np.outer(j, j) / n)
    assert np.allclose(oracle.fft1d(x, sign), F @ x, rtol=0, atol=1e-13 * max(1, n))


def test_fft1d_roundtrip_parseval_delta():
    rng = np.random.default_rng(1)
    n = 128
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = oracle.fft1d(x, -1)
    assert np.allclose(oracle.fft1d(y, +1) / n, x, atol=1e-14)
    assert np.isclose(np.vdot(y, y).real, n * np.vdot(x, x).real, rtol=1e-13)
    d = np.zeros(n, complex)
    d[5] = 1
    assert np.allclose(oracle.fft1d(d, +1), np.exp(2j * np.pi * 5 * np.arange(n) / n), atol=1e-14)


def test_fft3d_vs_numpy():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((8, 16, 4)) + 1j * rng.standard_normal((8, 16, 4))
    assert np.allclose(oracle.fft3d(x, -1), np.fft.fftn(x), atol=1e-12)
    assert np.allclose(oracle.fft3d(x, +1), np.fft.ifftn(x) * x.size, atol=1e-12)


# ---------------------------------------------------------------- potential

def test_vtilde_vs_numpy_fft():
    rng = np.random.default_rng(3)
    v = rng.standard_normal((12, 10, 8))
    K = (3, 4, 2)
    vt = oracle.vtilde(v, K)
    ref = np.fft.fftn(v) / v.size
    for k1, k2, k3 in itertools.product(*[range(-k, k + 1) for k in K]):
        assert abs(vt[k1 + K[0], k2 + K[1], k3 + K[2]] - ref[k1, k2, k3]) < 1e-14


def test_vtilde_closed_forms():
    N = (9, 8, 10)
    j = np.indices(N)
    k0, phi, amp = (2, -1, 3), 0.37, 0.8
    arg = 2 * np.pi * sum(k0[d] * j[d] / N[d] for d in range(3)) + phi
    v = 2 * amp * np.cos(arg) + 1.5
    K = (3, 3, 3)
    vt = oracle.vtilde(v, K)
    expect = np.zeros_like(vt)
    expect[K] = 1.5
    expect[tuple(np.add(k0, K))] = amp * np.exp(1j * phi)
    expect[tuple(np.add(np.negative(k0), K))] = amp * np.exp(-1j * phi)
    assert np.abs(vt - expect).max() < 1e-14


# ---------------------------------------------------------------- Hamiltonian

def _eig_via_apply(h):
    """Dense H assembled column by column through the FFT apply."""
    Hc = h.apply(np.eye(h.ng, dtype=complex)).T
    return Hc


def test_free_electron_eigenvalues():
    a, ecut, g = 6.0, 4.0, 16
    cell = np.eye(3) * a
    h = oracle.Hamiltonian(cell, ecut, np.zeros((g, g, g)))
    mil, _ = oracle.sphere(cell, ecut)
    kin = 0.5 * np.sum((mil * (2 * np.pi / a)) ** 2, axis=1)
    H = _eig_via_apply(h)
    assert np.abs(H - np.diag(kin)).max() < 1e-13
    assert np.allclose(h.kin, kin, rtol=1e-15, atol=1e-15)


def test_constant_potential_shift():
    a, ecut, g, c0 = 6.0, 4.0, 16, -0.731
    h = oracle.Hamiltonian(np.eye(3) * a, ecut, np.full((g, g, g), c0))
    H = _eig_via_apply(h)
    assert np.abs(H - np.diag(h.kin + c0)).max() < 1e-13


def test_cosine_potential_matrix_elements():
    # V(r) = 2 v cos(2 pi k0.j/N + phi): H_loc[m, n] = v e^{+i phi} when
    # n_m - n_n = k0 (pins the Fourier sign convention of (e2) and (e5))
    a, ecut, g = 6.0, 4.0, 18
    j = np.indices((g, g, g))
    k0, phi, amp = np.array([1, 0, -2]), 0.4, 0.3
    v = 2 * amp * np.cos(2 * np.pi * (k0[:, None, None, None] * j).sum(0) / g + phi)
    h = oracle.Hamiltonian(np.eye(3) * a, ecut, v)
    H = _eig_via_apply(h) - np.diag(h.kin)
    mil = h.miller
    index = {tuple(m): i for i, m in enumerate(mil)}
    expect = np.zeros_like(H)
    for n, mn in enumerate(mil):
        for sgn, val in ((1, amp * np.exp(1j * phi)), (-1, amp * np.exp(-1j * phi))):
            m = index.get(tuple(mn + sgn * k0))
            if m is not None:
                expect[m, n] = val
    assert np.abs(H - expect).max() < 1e-14


def test_dense_equals_apply_and_hermitian():
    spec, c, v, h = tiny(seed=1)
    H = h.dense()
    Ha = _eig_via_apply(h)
    assert np.abs(H - Ha).max() < 1e-13
    assert np.abs(H - H.conj().T).max() < 1e-14
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, h.ng)) + 1j * rng.standard_normal((2, h.ng))
    hx = h.apply(x)
    assert abs(np.vdot(x[0], hx[1]) - np.conj(np.vdot(x[1], hx[0]))) < 1e-12


def test_projectors_normalised_and_time_reversal():
    spec, c, v, h = tiny(seed=2)
    B = h.beta
    assert np.allclose(np.sum(np.abs(B) ** 2, axis=1), 1.0, atol=1e-14)
    mil = h.miller
    index = {tuple(m): i for i, m in enumerate(mil)}
    minus = np.array([index[tuple(-m)] for m in mil])
    assert np.abs(B[:, minus] - B.conj()).max() < 1e-15
    # s and p of one atom are orthogonal on the centrosymmetric sphere
    assert abs(np.vdot(B[0], B[1])) < 1e-14


def test_single_projector_secular_equation():
    # V = 0 plus one s projector: H = T + D beta beta^H, whose eigenvalues
    # off the kinetic spectrum solve 1 = D sum_G |beta_G|^2 / (lam - kin_G)
    a, ecut, g = 6.0, 3.0, 16
    proj = [dict(center=np.array([1.1, 2.3, 0.4]), l=0, m=0, width=0.7, d=-0.9)]
    h = oracle.Hamiltonian(np.eye(3) * a, ecut, np.zeros((g, g, g)), proj)
    w = np.linalg.eigvalsh(_eig_via_apply(h))
    kin, b2 = h.kin, np.abs(h.beta[0]) ** 2
    shells = np.unique(np.round(kin, 10))
    off = [lam for lam in w if np.min(np.abs(shells - lam)) > 1e-6]
    assert len(off) == len(shells)  # one secular root per distinct shell
    for lam in off:
        f = 1 - proj[0]["d"] * np.sum(b2 / (lam - kin))
        assert abs(f) < 1e-9
    assert off[0] < 0  # D < 0 binds one state below zero


def test_translation_invariance():
    # shift every well and projector by a grid vector: the spectrum is unchanged
    spec = synth.small_cell(a=6.0, ecut=3.5, grid=16, n_atoms=2)
    c, v = cell_data(spec, seed=4)
    h0 = oracle.Hamiltonian(c["cell"], c["ecut"], v, c["projectors"])
    s = np.array([3, -5, 7])
    shift = s * spec.a / spec.grid
    v1 = synth.vloc_on_grid(c["cell"], c["grid"], c["positions"] + shift, c["depths"], c["widths"])
    assert np.abs(v1 - np.roll(v, s, axis=(0, 1, 2))).max() < 1e-12
    proj1 = [dict(p, center=p["center"] + shift) for p in c["projectors"]]
    h1 = oracle.Hamiltonian(c["cell"], c["ecut"], v1, proj1)
    w0 = np.linalg.eigvalsh(h0.dense())
    w1 = np.linalg.eigvalsh(h1.dense())
    assert np.abs(w0 - w1).max() < 1e-12
    # the opposite projector phase would break this: exp(+iG.R) is not a symmetry
    proj2 = [dict(p, center=p["center"] - shift) for p in c["projectors"]]
    w2 = np.linalg.eigvalsh(oracle.Hamiltonian(c["cell"], c["ecut"], v1, proj2).dense())
    assert np.abs(w0 - w2).max() > 1e-4


# ---------------------------------------------------------------- small dense

@pytest.mark.parametrize("n", [1, 2, 5, 17, 40])
def test_jacobi_heev_vs_lapack(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = A + A.conj().T
    w, V, _ = oracle.heev(A)
    assert np.allclose(w, np.linalg.eigvalsh(A), atol=1e-12)
    assert np.abs(A @ V - V * w).max() < 1e-12
    assert np.abs(V.conj().T @ V - np.eye(n)).max() < 1e-13


def test_jacobi_degenerate_spectrum():
    rng = np.random.default_rng(9)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12)))
    d = np.array([1, 1, 1, 2, 2, 3, 4, 4, 4, 4, 5, 6], float)
    A = (Q * d) @ Q.conj().T
    w, V, _ = oracle.heev(A)
    assert np.allclose(w, d, atol=1e-13)
    assert np.abs(V.conj().T @ V - np.eye(12)).max() < 1e-13


def test_cholesky_vs_lapack():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((20, 20)) + 1j * rng.standard_normal((20, 20))
    S = X @ X.conj().T + 0.1 * np.eye(20)
    rc, L = oracle.cholesky(S)
    assert rc == 0
    assert np.allclose(L, np.linalg.cholesky(S), atol=1e-12)
    S[3] = S[4]
    S[:, 3] = S[:, 4]
    assert oracle.cholesky(S)[0] == -1


# ---------------------------------------------------------------- preconditioner

def test_teter_limits():
    assert oracle.teter(0.0) == 1.0
    xs = np.linspace(0, 50, 501)
    k = np.array([oracle.teter(x) for x in xs])
    assert np.all(np.diff(k) < 0) and np.all(k > 0)
    # large-x tail 8x^3 / 16x^4 = 1/(2x)
    assert abs(oracle.teter(1e4) * 2e4 - 1) < 1e-3


@pytest.mark.parametrize("x,num,den", [(1, 65, 81), (2, 175, 431), (0.5, 40, 41), (3, 405, 1701), (0.25, 518, 519)])
def test_teter_exact_rationals(x, num, den):
    """The Teter-Payne-Allan polynomial ratio (PRB 40, 12255) at points where it
    is a small exact fraction, worked by hand: x = 1 gives 65/81, x = 2 gives
    175/431, x = 1/2 gives (27 + 9 + 3 + 1)/(40 + 1) = 40/41, x = 3 gives
    405/1701, x = 1/4 gives 518/519 (numerator 27 + 4.5 + 0.75 + 0.125, the x^4
    term 16/256, both times 16).  Each coefficient 27, 18, 12, 8, 16 moves at least one of
    these values."""
    assert abs(oracle.teter(x) - num / den) <= 2e-16 * (num / den)


def test_residual_norms_against_numpy_and_dense_h():
    """|H psi_b - eps_b psi_b|: the oracle routine against numpy on random
    blocks (with a non-contiguous shift pattern), and the residual history of
    a ParO run against a recomputation from the dense matrix of H."""
    rng = np.random.default_rng(11)
    psi = rng.standard_normal((7, 513)) + 1j * rng.standard_normal((7, 513))
    hpsi = rng.standard_normal((7, 513)) + 1j * rng.standard_normal((7, 513))
    eps = rng.uniform(-2, 2, 7)
    ref = np.linalg.norm(hpsi - eps[:, None] * psi, axis=1)
    assert np.allclose(oracle.residual_norms(psi, hpsi, eps), ref, rtol=1e-14, atol=0)
    # an exact eigenpair of a diagonal operator has zero residual
    d = rng.uniform(0, 1, 513)
    e0 = np.zeros((1, 513), complex)
    e0[0, 17] = 1j
    assert oracle.residual_norms(e0, d[None, :] * e0, d[17:18])[0] == 0.0
    spec, c, v, h = tiny(seed=2)
    H = h.dense()
    x = synth.trial_block(h.ng, 4, 2)
    out = h.paro(x, 2, 6, h.shift_bound())
    r = np.linalg.norm(out["psi"] @ H.T - out["eps"][:, None] * out["psi"], axis=1)
    assert np.allclose(out["res_hist"][-1], r, rtol=1e-9, atol=1e-13)


# ---------------------------------------------------------------- PCG

def test_pcg_converges_to_direct_solve():
    spec, c, v, h = tiny(seed=3, a=5.0, ecut=2.5, grid=16)
    H = h.dense()
    lam = np.linalg.eigvalsh(H)
    sigma = h.shift_bound()
    assert sigma < lam[0]
    rng = np.random.default_rng(7)
    nb = 3
    psi = rng.standard_normal((nb, h.ng)) + 1j * rng.standard_normal((nb, h.ng))
    psi /= np.linalg.norm(psi, axis=1)[:, None]
    hpsi = psi @ H.T
    eps = np.einsum("bg,bg->b", psi.conj(), hpsi).real
    u, flags, gh = h.pcg(psi, hpsi, eps, sigma, h.ng, gamma_hist=True)
    A = H - sigma * np.eye(h.ng)
    for b in range(nb):
        ref = np.linalg.solve(A, (eps[b] - sigma) * psi[b])
        assert np.linalg.norm(u[b] - ref) < 1e-9 * np.linalg.norm(ref)
    assert not flags.any()


def test_pcg_exact_eigenvector_is_fixed_point():
    spec, c, v, h = tiny(seed=3, a=5.0, ecut=2.5, grid=16)
    H = h.dense()
    lam, Vec = np.linalg.eigh(H)
    psi = Vec[:, :2].T.copy()
    hpsi = psi @ H.T
    u, flags = h.pcg(psi, hpsi, lam[:2], h.shift_bound(), 10)
    assert np.abs(u - psi).max() < 1e-11


def test_projected_correction_solves_the_projected_system():
    """Algorithm 3, step 3: with n_cg = n_g the projected PCG gives the solution
    of (I - P)(H - sigma)(I - P) e = (eps - H) psi on the complement of psi,
    computed independently in an orthonormal basis Q of that complement:
    e = Q (Q^H (H - sigma) Q)^-1 Q^H (eps psi - H psi)."""
    spec, c, v, h = tiny(seed=3, a=5.0, ecut=2.5, grid=16)
    H = h.dense()
    sigma = h.shift_bound()
    rng = np.random.default_rng(11)
    nb = 3
    psi = rng.standard_normal((nb, h.ng)) + 1j * rng.standard_normal((nb, h.ng))
    psi /= np.linalg.norm(psi, axis=1)[:, None]
    hpsi = psi @ H.T
    eps = np.einsum("bg,bg->b", psi.conj(), hpsi).real
    e, flags = h.pcg(psi, hpsi, eps, sigma, h.ng, projected=True)
    assert not flags.any()
    A = H - sigma * np.eye(h.ng)
    for b in range(nb):
        # orthonormal basis of the complement of psi_b: trailing columns of a full QR
        Q, _ = np.linalg.qr(np.column_stack([psi[b], rng.standard_normal((h.ng, h.ng - 1))]), mode="complete")
        Q = Q[:, 1:]
        rhs = eps[b] * psi[b] - hpsi[b]
        ref = Q @ np.linalg.solve(Q.conj().T @ A @ Q, Q.conj().T @ rhs)
        assert np.linalg.norm(e[b] - ref) < 1e-9 * np.linalg.norm(ref)
        assert abs(np.vdot(psi[b], e[b])) < 1e-12 * np.linalg.norm(e[b])
        # not the unprojected correction of Algorithm 2
        e2 = np.linalg.solve(A, rhs)
        assert np.linalg.norm(e2 - ref) > 1e-3 * np.linalg.norm(ref)


def test_projected_correction_vanishes_at_an_eigenvector():
    spec, c, v, h = tiny(seed=3, a=5.0, ecut=2.5, grid=16)
    H = h.dense()
    lam, Vec = np.linalg.eigh(H)
    psi = Vec[:, :2].T.copy()
    e, flags = h.pcg(psi, psi @ H.T, lam[:2], h.shift_bound(), 10, projected=True)
    assert np.abs(e).max() < 1e-12


def test_pcg_negative_curvature_flag():
    spec, c, v, h = tiny(seed=3, a=5.0, ecut=2.5, grid=16)
    H = h.dense()
    lam, Vec = np.linalg.eigh(H)
    rng = np.random.default_rng(1)
    psi = rng.standard_normal((1, h.ng)) + 1j * rng.standard_normal((1, h.ng))
    hpsi = psi @ H.T
    # a shift far above the spectrum makes H - sigma negative definite
    u, flags = h.pcg(psi, hpsi, np.array([0.0]), lam[-1] + 1.0, 5)
    assert flags[0] & oracle.F_NEGCURV


# ---------------------------------------------------------------- Rayleigh-Ritz

def test_rayleigh_ritz_invariant_subspace_and_bounds():
    spec, c, v, h = tiny(seed=5)
    H = h.dense()
    lam, Vec = np.linalg.eigh(H)
    rng = np.random.default_rng(2)
    m = 6
    X = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    U = (Vec[:, :m] @ X).T.copy()                  # exact invariant subspace, mixed
    eps, psi, hpsi, f = oracle.rayleigh_ritz(U, U @ H.T, m)
    assert f == 0
    assert np.allclose(eps, lam[:m], atol=1e-12)
    assert np.abs(psi.conj() @ psi.T - np.eye(m)).max() < 1e-12
    assert np.abs(hpsi - psi @ H.T).max() < 1e-11
    # random subspace: Ritz values bound the eigenvalues from above
    U = rng.standard_normal((m, h.ng)) + 1j * rng.standard_normal((m, h.ng))
    eps, psi, hpsi, f = oracle.rayleigh_ritz(U, U @ H.T, m)
    assert np.all(eps >= lam[:m] - 1e-12)
    # invariance under U -> X U
    eps2, *_ = oracle.rayleigh_ritz(X @ U, X @ U @ H.T, m)
    assert np.allclose(eps, eps2, atol=1e-11)


def test_rayleigh_ritz_singular_overlap_falls_back():
    spec, c, v, h = tiny(seed=5)
    H = h.dense()
    lam, Vec = np.linalg.eigh(H)
    U = np.concatenate([Vec[:, :4].T, Vec[:, :4].T + 1e-9 * Vec[:, 4:8].T])
    eps, psi, hpsi, f = oracle.rayleigh_ritz(U, U @ H.T, 4)
    assert f & oracle.F_CHOL
    assert np.allclose(eps, lam[:4], atol=1e-10)


# ---------------------------------------------------------------- shift bound

def test_shift_bound_is_a_lower_bound():
    spec, c, v, h = tiny(seed=6)
    H = h.dense()
    B = h.beta
    D = np.array([p["d"] for p in c["projectors"]])
    vnl = (B.T * D) @ B.conj()
    assert abs(h.nl_min_eig() - min(0, np.linalg.eigvalsh(vnl)[0])) < 1e-12 \
        or h.nl_min_eig() >= 0
    assert abs(h.vmin - v.min()) == 0
    assert h.shift_bound() < np.linalg.eigvalsh(H)[0]


# ---------------------------------------------------------------- ParO loop

def test_paro_fixed_point():
    spec, c, v, h = tiny(seed=7)
    H = h.dense()
    lam, Vec = np.linalg.eigh(H)
    nb = 4
    r = h.paro(Vec[:, :nb].T.copy(), 2, 6, h.shift_bound())
    assert np.abs(r["eps_hist"] - lam[:nb]).max() < 1e-12
    P = Vec[:, :nb]
    Q = r["psi"].T
    sin = np.linalg.norm(Q - P @ (P.conj().T @ Q), 2)
    assert sin < 1e-10


def test_paro_converges_tiny_cell():
    spec, c, v, h = tiny(seed=8)
    lam = np.linalg.eigvalsh(h.dense())
    x = synth.trial_block(h.ng, 8, 8)
    r = h.paro(x, 40, 10, h.shift_bound(), variant=0, shift_mode=1)
    assert np.abs(r["eps"][:4] - lam[:4]).max() < 1e-9
    # eigenvalue errors never go negative (Ritz values are upper bounds)
    assert np.all(r["eps_hist"][:, :4] - lam[:4] > -1e-12)


def test_mparo2_converges_on_the_1503_plane_wave_cell():
    """Algorithm 3 (MParO II) reaches the dense eigenvalues like Algorithm 2."""
    spec = synth.WORKLOADS["c0"]
    c, v = cell_data(spec, 0)
    h = oracle.Hamiltonian(c["cell"], c["ecut"], v, c["projectors"])
    lam = np.linalg.eigvalsh(h.dense())
    x = synth.trial_block(h.ng, 16, 0)
    r = h.paro(x, 30, 10, h.shift_bound(), variant=2, shift_mode=1)
    err = np.abs(r["eps_hist"][:, :8] - lam[:8]).max(axis=1)
    assert err[-1] < 1e-8
    assert r["flags"] == 0


def test_mparo_converges_on_the_1503_plane_wave_cell():
    spec = synth.WORKLOADS["c0"]
    c, v = cell_data(spec, 0)
    h = oracle.Hamiltonian(c["cell"], c["ecut"], v, c["projectors"])
    lam = np.linalg.eigvalsh(h.dense())
    x = synth.trial_block(h.ng, 16, 0)
    r = h.paro(x, 30, 10, h.shift_bound(), variant=1, shift_mode=1)
    err = np.abs(r["eps_hist"][:, :8] - lam[:8]).max(axis=1)
    assert err[-1] < 1e-8
    assert r["flags"] == 0


# ---------------------------------------------------------------- density and the eigenvalue gradient

def _numpy_density(h, psi, w):
    """|inverse FFT|^2 of the coefficients scattered onto the grid (numpy's FFT)."""
    N = np.array(h.grid)
    mil = h.miller
    rho = np.zeros(h.grid)
    for b in range(psi.shape[0]):
        g = np.zeros(h.grid, complex)
        g[mil[:, 0] % N[0], mil[:, 1] % N[1], mil[:, 2] % N[2]] = psi[b]
        rho += w[b] * np.abs(np.fft.ifftn(g) * np.prod(N)) ** 2
    return rho


def test_density_vs_numpy_ifft_and_parseval():
    spec, c, v, h = tiny(seed=9)
    x = synth.trial_block(h.ng, 3, 9)
    w = np.array([2.0, 0.5, 1.25])
    rho = h.density(x, w)
    ref = _numpy_density(h, x, w)
    assert np.abs(rho - ref).max() < 1e-12 * ref.max()
    # Parseval: sum_j |psi(r_j)|^2 = N1 N2 N3 ||c||^2 (grid holds the sphere without aliasing)
    assert abs(rho.sum() - np.prod(h.grid) * (w * (np.abs(x) ** 2).sum(axis=1)).sum()) < 1e-10 * rho.sum()
    # default weights are one
    assert np.allclose(h.density(x), _numpy_density(h, x, np.ones(3)), rtol=0, atol=1e-12 * ref.max())


def test_density_of_single_plane_waves_is_uniform():
    """A plane wave has |psi|^2 = |c|^2 at every grid point, whatever its index."""
    spec, c, v, h = tiny(seed=10)
    x = np.zeros((3, h.ng), complex)
    x[0, 0] = 1.0
    x[1, h.ng // 2] = 0.6 - 0.8j
    x[2, h.ng - 1] = 2.0j
    rho = h.density(x, [1.0, 3.0, 0.25])
    assert np.abs(rho - (1.0 + 3.0 + 0.25 * 4.0)).max() < 1e-12
    # two plane waves: |a + b e^{2 pi i (n - n').j/N}|^2 is a cosine on the grid
    mil = h.miller
    x = np.zeros((1, h.ng), complex)
    x[0, 0], x[0, 5] = 1.0, 0.5
    rho = h.density(x)
    dn = mil[5] - mil[0]
    J = np.indices(h.grid).reshape(3, -1).T
    ph = 2 * np.pi * (J * (dn / np.array(h.grid))).sum(axis=1)
    ref = (1.25 + np.cos(ph)).reshape(h.grid)
    assert np.abs(rho - ref).max() < 1e-12


def test_density_is_the_hellmann_feynman_gradient_of_the_eigenvalue_sum():
    """Central differences of the lowest dense eigenvalues (LAPACK) with respect to
    V at single grid points equal rho_j / (N1 N2 N3) built from the eigenvectors."""
    spec, c, v, h = tiny(seed=11)
    lam, vec = np.linalg.eigh(h.dense())
    # k with a clear gap above it, so the weighted sum is differentiable
    k = next(k for k in range(4, 9) if lam[k] - lam[k - 1] > 1e-3)
    w = np.linspace(2.0, 1.0, k)
    rho = h.density(vec[:, :k].T.copy(), w)
    nv = np.prod(h.grid)
    rng = np.random.default_rng(11)
    pts = [tuple(rng.integers(0, g) for g in h.grid) for _ in range(4)]
    pts.append(tuple(int(i) for i in np.unravel_index(np.argmax(rho), h.grid)))
    step = 1e-3
    for j in pts:
        vals = []
        for s in (+step, -step):
            vp = v.copy()
            vp[j] += s
            hp = oracle.Hamiltonian(c["cell"], c["ecut"], vp, c["projectors"])
            vals.append(w @ np.linalg.eigvalsh(hp.dense())[:k])
        fd = (vals[0] - vals[1]) / (2 * step)
        assert abs(fd - rho[j] / nv) < 1e-8 * max(1.0, rho.max() / nv), (j, fd, rho[j] / nv)
    # and the mirrored point j -> -j does not match where the density is not symmetric
    jm = tuple((-np.array(pts[-1])) % np.array(h.grid))
    assert abs(rho[jm] - rho[pts[-1]]) > 1e-3 * rho.max()


def test_projector_gradient_is_the_hellmann_feynman_derivative():
    """Central differences of the lowest dense eigenvalues (LAPACK) with respect to
    every KB energy d_p and every projector centre component R_p equal the
    oracle's projector gradient built from the eigenvectors."""
    import copy
    spec, c, v, h = tiny(seed=12)
    lam, vec = np.linalg.eigh(h.dense())
    k = next(k for k in range(4, 9) if lam[k] - lam[k - 1] > 1e-3)
    w = np.linspace(2.0, 1.0, k)
    dd, dR = h.projector_gradient(vec[:, :k].T.copy(), w)
    assert dd.shape == (len(c["projectors"]),) and dR.shape == (len(c["projectors"]), 3)

    def energy(projs):
        hp = oracle.Hamiltonian(c["cell"], c["ecut"], v, projs)
        return w @ np.linalg.eigvalsh(hp.dense())[:k]

    # Richardson-extrapolated central differences: O(h^4) truncation
    def deriv(f, h=1e-4):
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        return (4 * d2 - d1) / 3

    def shifted(p, key, a, s):
        q = copy.deepcopy(c["projectors"])
        if key == "d":
            q[p]["d"] += s
        else:
            q[p]["center"] = np.array(q[p]["center"], float)
            q[p]["center"][a] += s
        return energy(q)

    scale = max(1.0, np.abs(dd).max())
    for p in range(len(c["projectors"])):
        assert abs(deriv(lambda s: shifted(p, "d", 0, s)) - dd[p]) < 1e-9 * scale, p
        for a in range(3):
            assert abs(deriv(lambda s: shifted(p, "R", a, s)) - dR[p, a]) < 1e-9 * scale, (p, a)
    # |P|^2 >= 0, and the derivative is not trivially zero
    assert np.all(dd >= 0) and np.abs(dR).max() > 1e-3
