"""MI355X-native solver for holographic optical tweezers (RS / GS / GSW).

Implements the hot path of Bianchi & Di Leonardo, "Real-time optical
micro-manipulation using optimized holograms generated on the GPU"
(arXiv:0907.4027) as hand-written HIP kernels for CDNA4 behind the C ABI in
include/hot.h.  This package only marshals arguments into that library.
"""
from ._lib import (HOT_EDEGENERATE, HOT_EDEVICE, HOT_EINVAL, HOT_ENOMEM, HOT_MAX_BATCH, HOT_MAX_SIDE,
                   HOT_MAX_TRAPS, HOT_OK, HOT_ONTHEFLY, HOT_SEPARABLE, HOT_STORED, HotError, hot_slm, hot_stats, load)

__all__ = ["Context", "Result", "TrapField", "trap_intensity_loss", "optimize_phase", "HotError", "hot_slm",
           "hot_stats", "load", "HOT_OK", "HOT_EINVAL", "HOT_ENOMEM", "HOT_EDEVICE", "HOT_EDEGENERATE",
           "HOT_ONTHEFLY", "HOT_STORED", "HOT_SEPARABLE", "HOT_MAX_TRAPS", "HOT_MAX_SIDE", "HOT_MAX_BATCH"]


def __getattr__(name):
    # torch-dependent parts load on first use, so the C ABI can be inspected without torch
    if name in ("Context", "Result"):
        from . import solver
        return getattr(solver, name)
    if name in ("TrapField", "trap_intensity_loss", "optimize_phase"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
