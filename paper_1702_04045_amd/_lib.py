"""ctypes declarations of libparo's C ABI (include/paro.h).

Argument marshalling only: every step of the computation runs in the
library's HIP kernels.  Loading fails loudly when libparo.so is missing.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libparo.so")

PARO_OK, PARO_EINVAL, PARO_EALIAS, PARO_ESIZE, PARO_EHIP, PARO_EUNSUP = 0, -1, -2, -3, -4, -5
F_NEGCURV, F_CHOL, F_NAN = 1, 2, 4
SHIFT_FIXED, SHIFT_ADAPTIVE = 0, 1
VARIANT_PARO, VARIANT_MPARO1, VARIANT_MPARO2 = 0, 1, 2
PREC_FP64, PREC_MIXED, PREC_MIXED_BF16 = 0, 1, 2
TUNE_FORCE = 1
K_STICK_INV, K_PLANE, K_STICK_FWD, K_GEMM_HN, K_GEMM_NN, K_PCG_UPDATE, K_DENSITY = 1, 2, 3, 4, 5, 6, 7

ERRORS = {PARO_EINVAL: "EINVAL", PARO_EALIAS: "EALIAS", PARO_ESIZE: "ESIZE", PARO_EHIP: "EHIP",
          PARO_EUNSUP: "EUNSUP"}


class ParoError(RuntimeError):
    def __init__(self, code, fn, msg):
        super().__init__(f"{fn}: {ERRORS.get(code, code)}: {msg}")
        self.code = code


class Projector(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("l", C.c_int32), ("m", C.c_int32), ("width", C.c_double),
                ("d", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("cell", C.c_double * 9), ("ecut", C.c_double), ("grid", C.c_int32 * 3), ("n_g", C.c_int64),
                ("miller", C.POINTER(C.c_int32)), ("vloc", C.POINTER(C.c_double)), ("n_proj", C.c_int32),
                ("proj", C.POINTER(Projector))]


class PlanInfo(C.Structure):
    _fields_ = [("n_g", C.c_int64), ("nmax", C.c_int32 * 3), ("grid", C.c_int32 * 3), ("n_sticks", C.c_int32),
                ("n_proj", C.c_int32), ("omega", C.c_double)]


class TuneResult(C.Structure):
    _fields_ = [("schedule", C.c_int32 * 2), ("bands", C.c_int32 * 2), ("ms", C.c_double * 2),
                ("ms_default", C.c_double * 2), ("candidates", C.c_int32), ("cached", C.c_int32)]


class IterOpts(C.Structure):
    _fields_ = [("n_outer", C.c_int32), ("n_cg", C.c_int32), ("n_conv", C.c_int32), ("shift_mode", C.c_int32),
                ("variant", C.c_int32), ("initial_rr", C.c_int32), ("sigma_lb", C.c_double),
                ("tol_res", C.c_double), ("precision", C.c_int32)]


_vp, _dp, _ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
_sz = C.c_size_t

SIGNATURES = {
    "paro_abi_version": (C.c_int32, []),
    "paro_last_error": (C.c_char_p, []),
    "paro_sphere_enumerate": (C.c_int32, [_dp, C.c_double, C.c_int64, _ip, C.POINTER(C.c_int64), _ip]),
    "paro_grid_size": (C.c_int32, [_ip, _ip]),
    "paro_plan_bytes": (C.c_int32, [C.POINTER(Problem), C.POINTER(_sz)]),
    "paro_plan_create": (C.c_int32, [C.POINTER(Problem), _vp, _sz, _vp, C.POINTER(_vp)]),
    "paro_plan_destroy": (C.c_int32, [_vp]),
    "paro_plan_set_stream": (C.c_int32, [_vp, _vp]),
    "paro_plan_get_info": (C.c_int32, [_vp, C.POINTER(PlanInfo)]),
    "paro_plan_set_schedule": (C.c_int32, [_vp, C.c_int32, C.c_int32, C.c_int32]),
    "paro_plan_get_schedule": (C.c_int32, [_vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                           C.POINTER(C.c_int32)]),
    "paro_plan_autotune": (C.c_int32, [_vp, C.c_int32, _vp, C.c_size_t, C.c_int32, C.POINTER(TuneResult)]),
    "paro_workspace_bytes": (C.c_int32, [_vp, C.c_int32, C.POINTER(_sz)]),
    "paro_get_kinetic": (C.c_int32, [_vp, _vp]),
    "paro_get_projectors": (C.c_int32, [_vp, _vp]),
    "paro_apply_h": (C.c_int32, [_vp, C.c_int32, _vp, C.c_int64, _vp, _vp, _vp, _sz]),
    "paro_apply_h_f32": (C.c_int32, [_vp, C.c_int32, _vp, C.c_int64, _vp, _vp, _vp, _sz]),
    "paro_apply_h_f32_bf16": (C.c_int32, [_vp, C.c_int32, _vp, C.c_int64, _vp, _vp, _vp, _sz]),
    "paro_iterate_batch": (C.c_int32, [C.c_int32, C.POINTER(_vp), C.POINTER(C.c_int32), C.POINTER(_vp),
                                       C.POINTER(_vp), C.POINTER(C.c_int64), C.POINTER(_vp), C.POINTER(_vp),
                                       C.POINTER(IterOpts), C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_sz),
                                       C.POINTER(C.c_int32)]),
    "paro_density_workspace_bytes": (C.c_int32, [_vp, C.c_int32, C.POINTER(_sz)]),
    "paro_density": (C.c_int32, [_vp, C.c_int32, _vp, C.c_int64, _vp, _vp, _vp, _sz]),
    "paro_projector_gradient_workspace_bytes": (C.c_int32, [_vp, C.c_int32, C.POINTER(_sz)]),
    "paro_projector_gradient": (C.c_int32, [_vp, C.c_int32, _vp, C.c_int64, _vp, _vp, _vp, _vp, _sz]),
    "paro_source_solve": (C.c_int32, [_vp, C.c_int32, _vp, _vp, C.c_int64, _vp, _vp, C.c_int32, _vp, _vp, _vp,
                                      _sz]),
    "paro_source_solve_mixed": (C.c_int32, [_vp, C.c_int32, _vp, _vp, C.c_int64, _vp, _vp, C.c_int32, _vp, _vp, _vp,
                                      _sz]),
    "paro_rayleigh_ritz": (C.c_int32, [_vp, C.c_int32, C.c_int32, _vp, _vp, C.c_int64, _vp, _vp, _vp, _vp, _sz]),
    "paro_residual_norms": (C.c_int32, [_vp, C.c_int32, _vp, _vp, C.c_int64, _vp, _vp, _vp, _sz]),
    "paro_shift_lower_bound": (C.c_int32, [_vp, _vp, _vp, _sz]),
    "paro_iterate": (C.c_int32, [_vp, C.c_int32, _vp, _vp, C.c_int64, _vp, _vp, C.POINTER(IterOpts), _vp, _vp,
                                 _sz, _ip]),
    "paro_get_status": (C.c_int32, [_vp, _ip]),
    "paro_zgemm_hn": (C.c_int32, [_vp, C.c_int32, C.c_int32, C.c_int64, _vp, C.c_int64, _vp, C.c_int64, _vp,
                                  C.c_int64, _vp, _sz]),
    "paro_zgemm_nn": (C.c_int32, [_vp, C.c_int64, C.c_int32, C.c_int32, _vp, C.c_int64, _vp, C.c_int64, _vp,
                                  C.c_int64, C.c_int32]),
    "paro_zgemm_hn_noalloc": (C.c_int32, [_vp, C.c_int32, C.c_int32, C.c_int64, _vp, C.c_int64, _vp, C.c_int64,
                                          _vp, C.c_int64]),
    "paro_truncated_gradient_workspace_bytes": (C.c_int32, [_vp, C.c_int32, C.c_int32, C.c_int32, C.POINTER(_sz)]),
    "paro_truncated_gradient": (C.c_int32, [_vp, C.c_int32, _vp, C.c_int64, C.c_double, C.c_int32, C.c_int32, _vp,
                                            _vp, _vp, _vp, _vp, _sz]),
    "paro_profile_start": (C.c_int32, [C.c_int32, C.c_int32]),
    "paro_profile_start_sampled": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32]),
    "paro_profile_stop": (C.c_int32, [_ip, C.POINTER(C.c_double)]),
    "paro_heev_workspace_bytes": (C.c_int32, [C.c_int32, C.POINTER(_sz)]),
    "paro_heev": (C.c_int32, [_vp, C.c_int32, _vp, _vp, _vp, _vp, _sz]),
}

_lib = None


def load():
    """Load libparo.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1702_04045_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(rc, fn):
    if rc != PARO_OK:
        msg = load().paro_last_error()
        raise ParoError(rc, fn, msg.decode() if msg else "")
