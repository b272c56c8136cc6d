"""Host-side measurement helpers of bench.py (no GPU): the certified
eigenvalue-error bound and the algorithmic work counts of H psi."""
import numpy as np

import bench


def _ritz(H, X):
    """Rayleigh-Ritz on the column span of X (numpy): Ritz values, residual norms."""
    Q, _ = np.linalg.qr(X)
    w, Y = np.linalg.eigh(Q.conj().T @ H @ Q)
    V = Q @ Y
    return w, np.linalg.norm(H @ V - V * w, axis=0)


def test_kato_temple_bound_holds_and_is_quadratic():
    """On a Hermitian matrix with a known spectrum, Ritz pairs from perturbed
    eigenvectors: the bound is never below the true error max |eps_i - lambda_i|,
    and it falls quadratically with the residual (10x smaller perturbation,
    about 100x smaller bound) while |r| itself falls only linearly."""
    rng = np.random.default_rng(4)
    n, k = 200, 12
    lam = np.concatenate([np.linspace(-1.0, 0.0, k), np.sort(rng.uniform(0.5, 3.0, n - k))])
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    H = (Q * lam) @ Q.conj().T
    bounds, resmax = [], []
    for delta in (1e-3, 1e-4, 1e-5):
        X = Q[:, :k] + delta * (rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k)))
        w, r = _ritz(H, X)
        err = np.abs(w[:8] - lam[:8]).max()
        b = bench.kato_temple_bound(w, r, 8)
        assert b >= err
        bounds.append(b)
        resmax.append(r[:8].max())
    assert bounds[1] < bounds[0] / 30 and bounds[2] < bounds[1] / 30
    assert resmax[2] > resmax[0] / 300


def test_kato_temple_bound_falls_back_to_residual_without_gap():
    """A neighbour whose residual swallows the gap leaves only |r_i|."""
    eps = np.array([0.0, 0.01, 1.0])
    res = np.array([1e-3, 0.05, 1e-3])
    assert bench.kato_temple_bound(eps, res, 1) == 1e-3
    res2 = np.array([1e-3, 1e-4, 1e-3])
    assert abs(bench.kato_temple_bound(eps, res2, 1) - 1e-6 / (0.01 - 1e-4)) < 1e-18


def test_hpsi_work_counts():
    """Pruned transform lines of the 96^3 benchmark cell: 1281 z-sticks, 41
    populated columns per plane, 96 rows per plane, 5 N log2 N flops each way."""
    local, nl, byts = bench.hpsi_work(96, 1281, 41, 34265, 128, 64)
    lines = 1281 + 96 * 41 + 96 * 96
    assert abs(local - (2 * lines * 5 * 96 * np.log2(96) + 2 * 96 ** 3 + 4 * 34265)) < 1
    assert nl == 16 * 34265 * 128
    assert byts == 32 * 34265 + 8 * 96 ** 3 / 64
