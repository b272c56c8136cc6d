"""GPU parity of the split-BF16 projector products (paro_apply_h_f32_bf16 and
the PREC_MIXED_BF16 source problems) against the CPU oracle.

Bar of the apply.  The local part is the FP32 apply's: max |diff| <= 2e-6
max |ref|.  In the nonlocal part V_NL x = sum_p d_p beta_p (beta_p^H x),
every real operand x is held as hi + lo (two BF16 values, |x - hi - lo| <=
2^-16 |x|) and a product as hi hi + hi lo + lo hi, within 3 x 2^-16 of the
exact one; accumulation is FP32.  With S_pb = sum_g |beta_p(g)| |x_b(g)|
and P_pb = beta_p^H x_b, the error of element (b, g) is then at most about
    3 x 2^-16 sum_p |d_p| |beta_p(g)| (S_pb + |P_pb|),
and the tests take 2^-14 (a third more) as the factor.

The solver tests check what the mixed-precision scheme promises: the FP64
Rayleigh-Ritz refines the source problems' FP32 (here BF16-product)
corrections, so the converged eigenvalues are those of the FP64 run.
"""
import numpy as np
import pytest

import synth
from bench import kato_temple_bound
from test_gpu_parity import C1, EIG_TOL, TINY, make_case, to_dev, to_np

pytestmark = pytest.mark.gpu

PROJ12 = synth.small_cell(a=8.0, ecut=6.0, grid=24, n_atoms=3)
EPS_BF16X3 = 2.0 ** -14


def nl_bound(c, h, x):
    """Elementwise bound of the split-BF16 error of V_NL x (nb x n_g)."""
    beta = h.beta
    d = np.array([p["d"] for p in c["projectors"]])
    ab = np.abs(beta)
    S = ab @ np.abs(x).T                # (nproj, nb)
    P = np.abs(beta.conj() @ x.T)       # (nproj, nb)
    return EPS_BF16X3 * ((np.abs(d)[:, None] * (S + P)).T @ ab)


def check_apply(c, h, pl, x, idx=None):
    got = to_np(pl.apply_h_f32(to_dev(x), bf16=True))
    xs = x if idx is None else x[idx]
    g = got if idx is None else got[idx]
    ref = h.apply(xs.astype(np.complex128))
    bound = 2e-6 * np.abs(ref).max() + nl_bound(c, h, xs.astype(np.complex128))
    assert np.all(np.abs(g - ref) <= bound), np.max(np.abs(g - ref) / bound)
    # and the split products are not the FP32 ones: the difference to the
    # FP32 apply is of the split's order, not zero
    f32 = to_np(pl.apply_h_f32(to_dev(x)))
    f32 = f32 if idx is None else f32[idx]
    return np.abs(g - f32).max() / np.abs(ref).max()


@pytest.mark.parametrize("spec,nb", [(TINY, 3), (PROJ12, 37), (PROJ12, 1)], ids=["tiny", "p12_ragged37", "p12_1"])
def test_apply_h_f32_bf16_matches_oracle(spec, nb):
    """Ragged tiles: 8 or 12 projectors (one partial 32-row block), 37 bands
    (a partial 32-column block), a single band."""
    c, v, h, pl = make_case(spec, 4)
    x = synth.trial_block(h.ng, nb, 6).astype(np.complex64)
    d = check_apply(c, h, pl, x)
    assert 0 < d < 1e-3


def test_apply_h_f32_bf16_full_size_sampled_bands():
    """160 bands of the 34k-plane-wave cell with 128 projectors (many K splits
    of the B^H x product), three sampled against the oracle."""
    c, v, h, pl = make_case(C1, 0)
    x = synth.trial_block(h.ng, 160, 0).astype(np.complex64)
    check_apply(c, h, pl, x, idx=[0, 77, 159])


def test_bf16_padding_is_zero():
    """The zero padding of the split operands: a block whose trailing
    plane-wave coefficients are huge in the padded leading dimension gives
    the same result as the plain block (the pad is never read)."""
    import torch
    c, v, h, pl = make_case(PROJ12, 2)
    x = synth.trial_block(h.ng, 5, 1).astype(np.complex64)
    xd = torch.full((5, h.ng + 40), 1e30 + 1e30j, dtype=torch.complex64, device="cuda:0")
    xd[:, :h.ng] = to_dev(x)
    a = to_np(pl.apply_h_f32(xd, bf16=True))[:, :h.ng]
    b = to_np(pl.apply_h_f32(to_dev(x), bf16=True))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("variant", [0, 1], ids=["paro", "mparo"])
def test_mixed_bf16_reaches_dense_eigenvalues(variant):
    """ParO / MParO I with split-BF16 projector products in the FP32 source
    problems reach the dense eigenvalues of a 12-projector cell as the FP64
    run does, in at most two more outer iterations."""
    import paper_1702_04045_amd as P
    c, v, h, pl = make_case(PROJ12, 0)
    lam = np.linalg.eigvalsh(h.dense())
    runs = {}
    for prec in (P.PREC_FP64, P.PREC_MIXED_BF16):
        x = synth.trial_block(h.ng, 16, 0)
        runs[prec] = pl.iterate(to_dev(x), 80, 10, h.shift_bound(), variant=variant, shift_mode=1, n_conv=8,
                                tol_res=1e-7, precision=prec)
    eps = to_np(runs[P.PREC_MIXED_BF16]["eps"])
    assert runs[P.PREC_FP64]["n_done"] < 80
    assert np.abs(eps[:8] - lam[:8]).max() < 1e-8
    assert runs[P.PREC_MIXED_BF16]["n_done"] <= runs[P.PREC_FP64]["n_done"] + 2
    assert pl.status() == 0


def test_mixed_bf16_full_size_converges_to_fp64_eigenvalues():
    """The 34k-plane-wave cell at the benchmark shape (160 bands, 20 PCG
    steps, adaptive shift): the PREC_MIXED_BF16 run reaches a certified 1e-8 Ha
    bound for the 128 lowest bands, and its eigenvalues agree with the FP64
    run's to the FP64 bar."""
    import paper_1702_04045_amd as P
    c, v, h, pl = make_case(C1, 0)
    nb, nconv = C1.n_carried, C1.n_bands
    sig = pl.shift_lower_bound()
    final = {}
    for prec in (P.PREC_FP64, P.PREC_MIXED_BF16):
        out = pl.iterate(to_dev(synth.trial_block(h.ng, nb, 0)), 400, C1.n_cg, sig, shift_mode=1, n_conv=nconv,
                         tol_res=2e-6, precision=prec)
        st = to_np(out["stats"])[out["n_done"]]
        assert kato_temple_bound(st[:nb], st[nb:2 * nb], nconv) <= 1e-8
        final[prec] = to_np(out["eps"])[:nconv]
    a, b = final[P.PREC_FP64], final[P.PREC_MIXED_BF16]
    assert np.abs(a - b).max() <= EIG_TOL * max(1.0, np.abs(a).max())
    assert pl.status() == 0
