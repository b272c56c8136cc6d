"""Batched ParO (paro_iterate_batch) on cells of uneven grid, sphere and band
count: every cell's result is bitwise the one paro_iterate gives for that
cell alone, and one cell is checked against the oracle's ParO histories.
Batches of Algorithm 1 or 2 in FP64 or in mixed precision with FP32
projector products run their source problems as grouped launches (one
launch per kernel and FFT length for all cells, each cell's blocks
computing exactly what its own launch computes); MParO II and the split-BF16
mixed precision run cell by cell on the cells' streams.  Both paths are
covered.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def to_dev(x):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def to_np(t):
    return t.detach().cpu().numpy()


def small_specs():
    """Five cells: grids 16 to 48, 4 to 24 bands, with and without projectors."""
    return [
        synth.small_cell(a=6.0, ecut=4.0, grid=16, n_atoms=2, n_bands=4),
        synth.small_cell(a=8.0, ecut=6.0, grid=24, n_atoms=3, n_bands=9),
        synth.small_cell(a=9.0, ecut=8.0, grid=32, n_atoms=2, projectors=False, n_bands=16),
        synth.small_cell(a=7.0, ecut=5.0, grid=24, n_atoms=4, n_bands=5),
        synth.small_cell(a=11.0, ecut=9.0, grid=48, n_atoms=3, n_bands=24),
    ]


def build(specs, seed0=40):
    import paper_1702_04045_amd as P
    cells = []
    for i, sp in enumerate(specs):
        c = synth.make_cell(sp, seed0 + i)
        v = synth.vloc_on_grid(c["cell"], c["grid"], c["positions"], c["depths"], c["widths"])
        pl = P.Plan(c["cell"], c["ecut"], v, c["projectors"])
        x = synth.trial_block(pl.ng, sp.n_bands, seed0 + i)
        cells.append((sp, c, v, pl, x))
    return cells


@pytest.mark.parametrize("variant,shift_mode,tol,precision", [(0, 1, 0.0, 0), (1, 1, 1e-7, 0), (2, 0, 0.0, 0),
                                                               (1, 1, 0.0, 1), (0, 1, 1e-7, 1), (0, 1, 0.0, 2)],
                         ids=["paro_adaptive", "mparo_adaptive_tol", "mparo2_fixed", "mparo_mixed",
                              "paro_mixed_tol", "paro_mixed_bf16"])
def test_batch_is_bitwise_the_single_cell_runs(variant, shift_mode, tol, precision):
    import paper_1702_04045_amd as P
    torch = _torch()
    cells = build(small_specs())
    sig = [pl.shift_lower_bound() for _, _, _, pl, _ in cells]
    n_outer = 30 if tol > 0 else 12
    nconv = [max(1, sp.n_bands // 2) for sp, *_ in cells]
    ref = []
    for (sp, c, v, pl, x), s, k in zip(cells, sig, nconv):
        r = pl.iterate(to_dev(x), n_outer, 8, s, variant=variant, shift_mode=shift_mode, tol_res=tol, n_conv=k,
                       precision=precision)
        ref.append(r)
    psis = [to_dev(x) for *_, x in cells]
    got = P.iterate_batch([c[3] for c in cells], psis, n_outer, 8, sig, variant=variant, shift_mode=shift_mode,
                          tol_res=tol, n_conv=nconv, precision=precision,
                          streams=[torch.cuda.Stream() for _ in range(3)], stats=True)
    torch.cuda.synchronize()
    for k, (r, g) in enumerate(zip(ref, got)):
        assert g["n_done"] == r["n_done"], k
        assert torch.equal(g["psi"], r["psi"]), k
        assert torch.equal(g["eps"], r["eps"]), k
        assert torch.equal(g["hpsi"], r["hpsi"]), k
        assert torch.equal(g["sigma"], r["sigma"]), k
        rows = g["n_done"] + 1
        assert torch.equal(g["stats"][:rows], r["stats"][:rows]), k
    if tol > 0:
        assert len({g["n_done"] for g in got}) > 1  # cells stopped at their own iteration
    for _, _, _, pl, _ in cells:
        assert pl.status() == 0


def test_grouped_batch_many_cells_two_chunks_uneven_pcg_steps():
    """More entries than one grouped launch takes (70 cells, so the tables
    are split), a cell of 80 bands (two 64-band chunks of the stick and plane
    stages), cells with and without projectors, and three PCG step counts:
    every cell bitwise equal to its lone run."""
    import paper_1702_04045_amd as P
    torch = _torch()
    specs = [synth.small_cell(a=6.0, ecut=4.0, grid=16, n_atoms=2, n_bands=3 + i % 4,
                              projectors=(i % 3 != 0)) for i in range(69)]
    specs.append(synth.small_cell(a=10.0, ecut=8.0, grid=32, n_atoms=3, n_bands=80))
    cells = build(specs, seed0=70)
    sig = [pl.shift_lower_bound() for _, _, _, pl, _ in cells]
    ncg = [4 + i % 3 for i in range(len(cells))]
    ref = [pl.iterate(to_dev(x), 3, k, s, shift_mode=P.SHIFT_ADAPTIVE)
           for (sp, c, v, pl, x), s, k in zip(cells, sig, ncg)]
    got = P.iterate_batch([c[3] for c in cells], [to_dev(c[4]) for c in cells], 3, ncg, sig,
                          shift_mode=P.SHIFT_ADAPTIVE, streams=[torch.cuda.Stream() for _ in range(4)])
    torch.cuda.synchronize()
    for k, (r, g) in enumerate(zip(ref, got)):
        assert torch.equal(g["psi"], r["psi"]) and torch.equal(g["eps"], r["eps"]), k
        assert torch.equal(g["hpsi"], r["hpsi"]) and torch.equal(g["sigma"], r["sigma"]), k
    for _, _, _, pl, _ in cells:
        assert pl.status() == 0


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_captured_batch_replays_like_eager_runs(precision):
    """Fixed-shift outer iterations of a grouped batch captured into a graph
    (no host decisions): two replays, with other eager work between them,
    equal two eager batch calls from the same state bitwise."""
    import paper_1702_04045_amd as P
    torch = _torch()
    cells = build(small_specs(), seed0=90)
    plans = [c[3] for c in cells]
    sig = [pl.shift_lower_bound() for pl in plans]
    first = P.iterate_batch(plans, [to_dev(c[4]) for c in cells], 0, 8, sig, initial_rr=True)
    clone = lambda key: [o[key].clone() for o in first]  # noqa: E731
    ge, he, ee = clone("psi"), clone("hpsi"), clone("eps")
    gg, hg, eg = clone("psi"), clone("hpsi"), clone("eps")
    g = P.capture_batch(plans, gg, hg, eg, 3, 8, sig, precision=precision)
    for rep in range(2):
        g.replay()
        P.iterate_batch(plans, ge, 3, 8, sig, initial_rr=False, hpsis=he, epss=ee, precision=precision)
        torch.cuda.synchronize()
        for k in range(len(cells)):
            assert torch.equal(gg[k], ge[k]) and torch.equal(hg[k], he[k]) and torch.equal(eg[k], ee[k]), (rep, k)
        # unrelated eager work between the replays
        plans[0].iterate(to_dev(cells[0][4]), 2, 4, sig[0])
    for pl in plans:
        assert pl.status() == 0


def test_batch_cell_matches_oracle():
    """A cell with projectors inside a batch against the oracle's fixed-shift ParO histories."""
    import paper_1702_04045_amd as P
    torch = _torch()
    cells = build(small_specs()[:3], seed0=50)
    sp, c, v, pl, x = cells[1]
    h = oracle.Hamiltonian(c["cell"], c["ecut"], v, c["projectors"])
    sig = [p.shift_lower_bound() for _, _, _, p, _ in cells]
    sig[1] = h.shift_bound()
    got = P.iterate_batch([q[3] for q in cells], [to_dev(q[4]) for q in cells], 6, 8, sig, stats=True)
    torch.cuda.synchronize()
    r = h.paro(x, 6, 8, h.shift_bound(), variant=0, shift_mode=0)
    nb = sp.n_bands
    eps_hist = to_np(got[1]["stats"])[:, :nb]
    assert np.abs(eps_hist - r["eps_hist"]).max() < 1e-10 * max(1.0, np.abs(r["eps_hist"]).max())


def test_batch_of_the_uneven_workload_shapes():
    """The 24-cell uneven workload (grids 32 to 80, 11 to 84 bands, 16 to 96
    projectors): two outer iterations batched over 8 streams equal the
    single-cell runs bitwise, and every Ritz block stays orthonormal."""
    import paper_1702_04045_amd as P
    torch = _torch()
    specs = synth.batch_specs(0)
    cells = []
    for i, sp in enumerate(specs):
        c = synth.make_cell(sp, i)
        v = synth.vloc_on_grid(c["cell"], c["grid"], c["positions"], c["depths"], c["widths"])
        pl = P.Plan(c["cell"], c["ecut"], v, c["projectors"])
        cells.append((pl, synth.trial_block(pl.ng, sp.n_bands, i)))
    sig = [pl.shift_lower_bound() for pl, _ in cells]
    got = P.iterate_batch([pl for pl, _ in cells], [to_dev(x) for _, x in cells], 2, 10, sig,
                          shift_mode=P.SHIFT_ADAPTIVE)
    torch.cuda.synchronize()
    for k in (0, 5, 11, 23):
        pl, x = cells[k]
        r = pl.iterate(to_dev(x), 2, 10, sig[k], shift_mode=P.SHIFT_ADAPTIVE)
        assert torch.equal(got[k]["psi"], r["psi"]) and torch.equal(got[k]["eps"], r["eps"]), k
    for k, g in enumerate(got):
        psi = g["psi"]
        G = (psi.conj() @ psi.T).cpu().numpy()
        assert np.abs(G - np.eye(psi.shape[0])).max() < 1e-10, k
        assert cells[k][0].status() == 0, k


def test_batch_argument_errors():
    import ctypes as C

    import paper_1702_04045_amd as P
    from paper_1702_04045_amd import _lib as L
    cells = build(small_specs()[:2], seed0=60)
    pls = [q[3] for q in cells]
    psis = [to_dev(q[4]) for q in cells]
    # one workspace for both cells
    nb = [p.shape[0] for p in psis]
    ws0 = pls[0].workspace(max(nb))
    ws1 = pls[1].workspace(max(nb))
    assert ws0[0].value != ws1[0].value
    n = 2
    hpsi = [p.clone() for p in psis]
    eps = [_torch().zeros(k, dtype=_torch().float64, device="cuda:0") for k in nb]
    sig = [_torch().zeros(1, dtype=_torch().float64, device="cuda:0") for _ in nb]
    opts = (L.IterOpts * n)(*[L.IterOpts(n_outer=1, n_cg=2, n_conv=k, shift_mode=0, variant=0, initial_rr=1,
                                         sigma_lb=-5.0, tol_res=0.0, precision=0) for k in nb])
    vp = lambda ts: (C.c_void_p * n)(*[t.data_ptr() for t in ts])  # noqa: E731
    args = lambda wsl, ldv: (n, (C.c_void_p * n)(*[p.h.value for p in pls]), (C.c_int32 * n)(*nb),  # noqa: E731
                             vp(psis), vp(hpsi), (C.c_int64 * n)(*ldv), vp(eps), vp(sig), opts, None,
                             (C.c_void_p * n)(*[w[0].value for w in wsl]), (C.c_size_t * n)(*[w[1] for w in wsl]),
                             None)
    lib = P.load()
    assert lib.paro_iterate_batch(*args([ws0, ws0], [p.stride(0) for p in psis])) == L.PARO_EINVAL
    assert b"share a workspace" in lib.paro_last_error()
    assert lib.paro_iterate_batch(*args([ws0, ws1], [psis[0].stride(0), 1])) == L.PARO_EINVAL
    assert b"cell 1" in lib.paro_last_error()
    assert lib.paro_iterate_batch(0, *args([ws0, ws1], [p.stride(0) for p in psis])[1:]) == L.PARO_EINVAL
    _torch().cuda.synchronize()
