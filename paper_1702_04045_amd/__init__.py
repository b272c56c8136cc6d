"""MI355X (gfx950) hot path of the parallel orbital-updating (ParO) plane-wave eigensolver.

Pan, Dai, de Gironcoli, Gong, Rignanese, Zhou, arXiv 1702.04045.  The
numerical work lives in libparo.so (hand-written HIP, C ABI in
include/paro.h); this package only marshals arguments to it.
"""
from ._lib import (F_CHOL, F_NAN, F_NEGCURV, PREC_FP64, PREC_MIXED, PREC_MIXED_BF16, SHIFT_ADAPTIVE, SHIFT_FIXED, VARIANT_MPARO1,
                   VARIANT_MPARO2, VARIANT_PARO, ParoError, load)
from .paro import Plan, capture_batch, grid_size, heev, iterate_batch, sphere_enumerate, zgemm_hn, zgemm_hn_noalloc, zgemm_nn

__all__ = ["Plan", "iterate_batch", "capture_batch", "sphere_enumerate", "grid_size", "zgemm_hn", "zgemm_hn_noalloc", "zgemm_nn", "heev", "load", "ParoError",
           "F_NEGCURV", "F_CHOL", "F_NAN", "SHIFT_FIXED", "SHIFT_ADAPTIVE", "VARIANT_PARO", "VARIANT_MPARO1", "VARIANT_MPARO2",
           "PREC_FP64", "PREC_MIXED", "PREC_MIXED_BF16"]
