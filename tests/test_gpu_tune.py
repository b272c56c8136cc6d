"""The plane stage's selectable launch choices and the autotuner.

Every line schedule of every Stockham grid (24 to 80 points) and the three
of the 96-point grid, with several bands per work-group, against the oracle in
FP64 (1e-12) and FP32 (2e-6);
bands per work-group leave results bitwise unchanged; a schedule switch
re-lays the potential exactly (switching back restores bitwise results);
the autotuner picks a timed candidate no slower than the default and its
plan still matches the oracle; a batch whose cells use different schedules
on one grid is bitwise the cells' lone runs.
"""
import numpy as np
import pytest

import synth
from test_gpu_parity import make_case, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu

# cells whose largest Miller index is the largest the grid admits (N >= 4 m + 1)
EDGE = {24: 6.5, 32: 12.0, 40: 19.0, 48: 28.0, 64: 50.0, 80: 78.0}


def edge_spec(n):
    return synth.small_cell(a=10.0, ecut=EDGE[n], grid=n, n_atoms=2)


@pytest.mark.parametrize("n", sorted(EDGE))
def test_every_schedule_matches_oracle(n):
    import paper_1702_04045_amd as P
    c, v, h, pl = make_case(edge_spec(n), 3)
    assert 4 * int(h.nmax.max()) + 1 <= n < 4 * int(h.nmax.max()) + 9
    info = pl.get_schedule(P.PREC_FP64)
    assert info == dict(schedule=0, bands=4, n_schedules=3)
    x = synth.trial_block(h.ng, 7, 3)
    x32 = x.astype(np.complex64)
    ref = h.apply(x)
    ref32 = h.apply(x32.astype(np.complex128))
    base = base32 = None
    for s in range(3):
        got = {}
        for b in (2, 16, 1):
            pl.set_schedule(P.PREC_FP64, s, b)
            pl.set_schedule(P.PREC_MIXED, s, b)
            assert pl.get_schedule(P.PREC_FP64)["schedule"] == s and pl.get_schedule(P.PREC_MIXED)["bands"] == b
            g = to_np(pl.apply_h(to_dev(x)))
            g32 = to_np(pl.apply_h_f32(to_dev(x32)))
            assert rel_err(g, ref) < 1e-12, (s, b)
            assert rel_err(g32, ref32) < 2e-6, (s, b)
            got[b] = (g, g32)
        # bands per work-group change nothing
        assert np.array_equal(got[2][0], got[16][0]) and np.array_equal(got[2][0], got[1][0])
        assert np.array_equal(got[2][1], got[16][1]) and np.array_equal(got[2][1], got[1][1])
        if s == 0:
            base, base32 = got[2]
        else:
            # another radix order: another kernel, other rounding
            assert not np.array_equal(got[2][0], base)
    # back to schedule 0: the potential is re-laid exactly
    pl.set_schedule(P.PREC_FP64, 0, 4)
    pl.set_schedule(P.PREC_MIXED, 0, 4)
    assert np.array_equal(to_np(pl.apply_h(to_dev(x))), base)
    assert np.array_equal(to_np(pl.apply_h_f32(to_dev(x32))), base32)
    assert pl.status() == 0


@pytest.mark.parametrize("sched", [1, 2], ids=["paired", "cc"])
@pytest.mark.parametrize("nmax_edge", [False, True], ids=["c1like", "nmax23"])
def test_96_point_schedules(nmax_edge, sched):
    """Schedules 1 (four lanes per line, two threads of the cross-lane
    schedule in each) and 2 (the compressed-column plane, one band's
    populated columns in LDS) at 96 points against the oracle and against
    schedule 0, on a cell with the largest Miller index the pruned lines
    allow (23) and on a smaller one; bands per work-group change nothing;
    back to schedule 0 the potential is unchanged."""
    import paper_1702_04045_amd as P
    spec = (synth.small_cell(a=20.0, ecut=27.0, grid=96, n_atoms=3) if nmax_edge
            else synth.small_cell(a=20.0, ecut=20.0, grid=96, n_atoms=3))
    c, v, h, pl = make_case(spec, 9)
    if nmax_edge:
        assert int(h.nmax.max()) == 23
    # a new 96-point plan: FP64 on schedule 2 with 2 bands per work-group
    assert pl.get_schedule(P.PREC_FP64) == dict(schedule=2, bands=2, n_schedules=3)
    assert pl.get_schedule(P.PREC_MIXED) == dict(schedule=0, bands=4, n_schedules=3)
    pl.set_schedule(P.PREC_FP64, 0, 4)
    x = synth.trial_block(h.ng, 37, 9)
    x32 = x.astype(np.complex64)
    ref = h.apply(x)
    ref32 = h.apply(x32.astype(np.complex128))
    base = to_np(pl.apply_h(to_dev(x)))
    base32 = to_np(pl.apply_h_f32(to_dev(x32)))
    got = {}
    for b in (4, 1, 16):
        pl.set_schedule(P.PREC_FP64, sched, b)
        pl.set_schedule(P.PREC_MIXED, sched, b)
        g = to_np(pl.apply_h(to_dev(x)))
        g32 = to_np(pl.apply_h_f32(to_dev(x32)))
        assert rel_err(g, ref) < 1e-12, b
        assert rel_err(g32, ref32) < 2e-6, b
        # the same operations as schedule 0 up to how the compiler fuses them
        assert rel_err(g, base) < 1e-14, b
        assert rel_err(g32, base32) < 1e-6, b
        got[b] = (g, g32)
    assert np.array_equal(got[4][0], got[1][0]) and np.array_equal(got[4][0], got[16][0])
    assert np.array_equal(got[4][1], got[1][1]) and np.array_equal(got[4][1], got[16][1])
    pl.set_schedule(P.PREC_FP64, 0, 4)
    pl.set_schedule(P.PREC_MIXED, 0, 4)
    assert np.array_equal(to_np(pl.apply_h(to_dev(x))), base)
    assert np.array_equal(to_np(pl.apply_h_f32(to_dev(x32))), base32)
    assert pl.status() == 0


def test_schedule_errors():
    import paper_1702_04045_amd as P
    _, _, _, p32 = make_case(edge_spec(32), 0)
    _, _, _, p96 = make_case(synth.small_cell(a=6.0, ecut=4.0, grid=96, n_atoms=2), 0)
    for pl, s, b, prec in ((p32, 3, 4, 0), (p32, -1, 4, 0), (p32, 0, 0, 0), (p32, 0, 65, 1), (p32, 0, 4, 7),
                           (p96, 3, 4, 0)):
        with pytest.raises(P.ParoError) as e:
            pl.set_schedule(prec, s, b)
        assert e.value.code == -1
    assert p96.get_schedule(P.PREC_MIXED) == dict(schedule=0, bands=4, n_schedules=3)
    # nothing changed by the refused calls
    assert p32.get_schedule(P.PREC_FP64) == dict(schedule=0, bands=4, n_schedules=3)


@pytest.mark.parametrize("n,nb", [(48, 37), (96, 70)])
def test_autotune_picks_a_timed_candidate(n, nb):
    import paper_1702_04045_amd as P
    spec = edge_spec(n) if n in EDGE else synth.small_cell(a=20.0, ecut=20.0, grid=96, n_atoms=3)
    c, v, h, pl = make_case(spec, 5)
    default = [pl.get_schedule(p) for p in (P.PREC_FP64, P.PREC_MIXED)]
    r = pl.autotune(nb, force=True)
    nsched = 3
    assert not r["cached"]
    assert r["candidates"] == nsched * 4
    for k in range(2):
        assert 0 <= r["schedule"][k] < nsched and r["bands"][k] in (2, 4, 8, 16)
        assert 0 < r["ms"][k] <= r["ms_default"][k]
        if (r["schedule"][k], r["bands"][k]) != (default[k]["schedule"], default[k]["bands"]):
            assert r["ms"][k] * 1.01 < r["ms_default"][k]
    assert pl.get_schedule(P.PREC_FP64)["schedule"] == r["schedule"][0]
    assert pl.get_schedule(P.PREC_MIXED)["bands"] == r["bands"][1]
    # the same shape again: the kept choice, no timing
    _, _, _, pl2 = make_case(spec, 5)
    r2 = pl2.autotune(nb)
    assert r2["cached"] and r2["schedule"] == r["schedule"] and r2["bands"] == r["bands"]
    x = synth.trial_block(h.ng, 5, 5)
    assert rel_err(to_np(pl2.apply_h(to_dev(x))), h.apply(x)) < 1e-12
    x32 = x.astype(np.complex64)
    assert rel_err(to_np(pl2.apply_h_f32(to_dev(x32))), h.apply(x32.astype(np.complex128))) < 2e-6
    assert pl.status() == 0 and pl2.status() == 0


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_batch_with_mixed_schedules_is_bitwise_the_lone_runs(precision):
    """Three cells on the 32-point grid with schedules 0, 1, 2 (and different
    bands per work-group), a 48-point cell with schedule 2 and two 96-point
    cells with schedules 1 and 2, in one grouped batch, against each cell's
    lone run."""
    import torch

    import paper_1702_04045_amd as P
    specs = [synth.small_cell(a=9.0, ecut=8.0, grid=32, n_atoms=2, n_bands=11),
             synth.small_cell(a=10.0, ecut=11.0, grid=32, n_atoms=3, n_bands=6),
             synth.small_cell(a=8.5, ecut=9.0, grid=32, n_atoms=2, n_bands=17),
             synth.small_cell(a=11.0, ecut=9.0, grid=48, n_atoms=3, n_bands=24),
             synth.small_cell(a=12.0, ecut=12.0, grid=96, n_atoms=2, n_bands=9),
             synth.small_cell(a=11.0, ecut=12.0, grid=96, n_atoms=2, n_bands=13)]
    cells = []
    for i, (sp, (s, b)) in enumerate(zip(specs, [(0, 4), (1, 2), (2, 16), (2, 8), (1, 4), (2, 2)])):
        c = synth.make_cell(sp, 70 + i)
        v = synth.vloc_on_grid(c["cell"], c["grid"], c["positions"], c["depths"], c["widths"])
        pl = P.Plan(c["cell"], c["ecut"], v, c["projectors"])
        pl.set_schedule(P.PREC_FP64, s, b)
        pl.set_schedule(P.PREC_MIXED, s, b)
        cells.append((pl, synth.trial_block(pl.ng, sp.n_bands, 70 + i)))
    sig = [pl.shift_lower_bound() for pl, _ in cells]
    ref = [pl.iterate(to_dev(x), 3, 6, s, precision=precision) for (pl, x), s in zip(cells, sig)]
    got = P.iterate_batch([pl for pl, _ in cells], [to_dev(x) for _, x in cells], 3, 6, sig, precision=precision)
    torch.cuda.synchronize()
    for k, (r, g) in enumerate(zip(ref, got)):
        assert torch.equal(g["psi"], r["psi"]) and torch.equal(g["eps"], r["eps"]), k
        assert torch.equal(g["hpsi"], r["hpsi"]), k
    for pl, _ in cells:
        assert pl.status() == 0
