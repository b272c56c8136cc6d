"""Event timing of one kernel class: every launch, or a sample of one in
`every`; the events are reused by the next profile; applies are unchanged
by the timing."""
import ctypes as C

import numpy as np
import pytest

import synth
from test_gpu_parity import make_case, to_dev, to_np

pytestmark = pytest.mark.gpu


def _profile(lib, L, pl, x, n_apply, every):
    import torch
    assert lib.paro_profile_start_sampled(L.K_PLANE, 64, every) == 0
    outs = [pl.apply_h(x) for _ in range(n_apply)]
    torch.cuda.synchronize()
    n, tot = C.c_int32(), C.c_double()
    assert lib.paro_profile_stop(C.byref(n), C.byref(tot)) == 0
    return n.value, tot.value, outs


def test_sampled_plane_timing():
    import paper_1702_04045_amd as P
    from paper_1702_04045_amd import _lib as L
    lib = P.load()
    c, v, h, pl = make_case(synth.small_cell(a=9.0, ecut=8.0, grid=32, n_atoms=2), 3)
    x = to_dev(synth.trial_block(h.ng, 70, 3))  # 70 bands: two plane launches per FP64 apply
    ref = to_np(pl.apply_h(x))
    # 5 applies, 10 launches: all of them, then launches 0, 3, 6, 9
    n1, t1, o1 = _profile(lib, L, pl, x, 5, 1)
    n3, t3, o3 = _profile(lib, L, pl, x, 5, 3)
    assert n1 == 10 and n3 == 4
    assert t1 > 0 and t3 > 0
    # a cap below the launches: the first `cap` sampled launches
    assert lib.paro_profile_start_sampled(L.K_PLANE, 2, 1) == 0
    for _ in range(3):
        pl.apply_h(x)
    n, tot = C.c_int32(), C.c_double()
    assert lib.paro_profile_stop(C.byref(n), C.byref(tot)) == 0 and n.value == 2
    for o in o1 + o3:
        assert np.array_equal(to_np(o), ref)
    # one profile at a time
    assert lib.paro_profile_start(L.K_PLANE, 4) == 0
    assert lib.paro_profile_start(L.K_PLANE, 4) == L.PARO_EINVAL
    assert lib.paro_profile_stop(None, None) == 0
    assert pl.status() == 0
