"""The allocation-free product paro_zgemm_hn_noalloc (fixed device scratch)
against paro_zgemm_hn (caller workspace) and numpy: two calls in a row, the
second smaller, so that the second runs on scratch the first has filled."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _case(M, N, K, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))
    B = rng.standard_normal((N, K)) + 1j * rng.standard_normal((N, K))
    return A, B


def test_noalloc_matches_workspace_product_twice():
    import torch
    import paper_1702_04045_amd as P
    for M, N, K, seed in [(160, 160, 34265, 1), (37, 21, 1000, 2)]:
        A, B = _case(M, N, K, seed)
        Ad, Bd = _dev(A), _dev(B)
        got = P.zgemm_hn_noalloc(Ad, Bd).cpu().numpy()
        ref = P.zgemm_hn(Ad, Bd).cpu().numpy()
        npy = (A.conj() @ B.T).T
        scale = np.abs(npy).max()
        assert np.abs(got - ref).max() <= 1e-13 * np.sqrt(K) * scale, (M, N, K)
        assert np.abs(got - npy).max() <= 1e-13 * np.sqrt(K) * scale, (M, N, K)
        torch.cuda.synchronize()


def test_noalloc_rejects_products_above_the_scratch():
    import paper_1702_04045_amd as P
    A, B = _case(2048, 2048, 4, 3)
    with pytest.raises(P.ParoError, match="scratch"):
        P.zgemm_hn_noalloc(_dev(A), _dev(B))
