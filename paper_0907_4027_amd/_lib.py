"""ctypes declarations of the C ABI in include/hot.h (argument marshalling only).

Loading fails loudly when the HIP library has not been built: there is no CPU
fallback anywhere in this package.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhot.so")

HOT_OK, HOT_EINVAL, HOT_ENOMEM, HOT_EDEVICE, HOT_EDEGENERATE = 0, -1, -2, -3, -4
HOT_ONTHEFLY, HOT_STORED, HOT_SEPARABLE = 0, 1, 2
HOT_MAX_TRAPS, HOT_MAX_SIDE, HOT_MAX_BATCH = 2048, 4096, 4096
HOT_TUNE_PIXELS_PER_LANE, HOT_TUNE_TRAPS_PER_LANE, HOT_TUNE_SEGMENT, HOT_TUNE_SLICES, HOT_TUNE_GRAPHS = 1, 2, 3, 4, 5
HOT_TUNE_SEP_WAVES, HOT_TUNE_SEP_CHUNK, HOT_TUNE_ROWS, HOT_TUNE_SEP_SPLIT, HOT_TUNE_FRACT = 6, 7, 8, 9, 10
HOT_REC_LDS, HOT_REC_SCALAR, HOT_REC_GLOBAL = 0, 1, 2
HOT_MAP_LINEAR, HOT_MAP_SQUARE = 0, 1

# every symbol include/hot.h declares
EXPORTS = ("hot_create", "hot_destroy", "hot_set_stream", "hot_set_variant", "hot_set_tuning", "hot_sync", "hot_check_problem",
           "hot_rs", "hot_gs", "hot_gsw", "hot_gsw_noalloc", "hot_gsw_batched", "hot_forward_V", "hot_adjoint", "hot_encode_u8", "hot_time_passes", "hot_pixel_pass_variant",
           "hot_probe_issue", "hot_probe_copy", "hot_last_error", "hot_abi_version")


class hot_slm(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("pitch", C.c_double), ("wavelength", C.c_double),
                ("focal", C.c_double)]


class hot_stats(C.Structure):
    _fields_ = [("efficiency", C.c_float), ("uniformity", C.c_float), ("sigma", C.c_float)]


class HotError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hot error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libhot.so and declare its signatures."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} is missing: run __graft_entry__.build() (or "
                          f"python -m paper_0907_4027_amd.build) first; there is no CPU fallback")
    lib = C.CDLL(path)
    P, i32, u64 = C.c_void_p, C.c_int32, C.c_uint64
    S = C.POINTER(hot_slm)
    ST = C.POINTER(hot_stats)
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int32)
    sig = {
        "hot_create": ([C.POINTER(P), C.c_int, P], C.c_int),
        "hot_destroy": ([P], C.c_int),
        "hot_set_stream": ([P, P], C.c_int),
        "hot_set_variant": ([P, C.c_int], C.c_int),
        "hot_set_tuning": ([P, C.c_int, C.c_int], C.c_int),
        "hot_sync": ([P], C.c_int),
        "hot_check_problem": ([S, i32, dp, i32], C.c_int),
        "hot_rs": ([P, S, i32, dp, dp, u64, P, P, ST], C.c_int),
        "hot_gs": ([P, S, i32, dp, dp, u64, i32, P, P, ST], C.c_int),
        "hot_gsw": ([P, S, i32, dp, dp, u64, i32, P, P, P, P, P, ST], C.c_int),
        "hot_gsw_noalloc": ([P, S, i32, dp, dp, u64, i32, P, P, P, P, P, ST], C.c_int),
        "hot_gsw_batched": ([P, S, i32, ip, dp, dp, i32, P, P, ST], C.c_int),
        "hot_forward_V": ([P, S, i32, ip, dp, P, P], C.c_int),
        "hot_adjoint": ([P, S, i32, ip, dp, P, P, P], C.c_int),
        "hot_encode_u8": ([P, C.c_int64, P, P], C.c_int),
        "hot_time_passes": ([P, S, i32, dp, dp, i32, P, P, C.POINTER(C.c_float)], C.c_int),
        "hot_pixel_pass_variant": ([P, S, i32, dp, dp, C.c_int, C.c_int, C.c_int, i32, P, C.POINTER(C.c_float)],
                                   C.c_int),
        "hot_probe_issue": ([P, C.c_int, C.c_int, C.c_int64, dp], C.c_int),
        "hot_probe_copy": ([P, P, P, C.c_int64, C.c_int, dp], C.c_int),
        "hot_last_error": ([], C.c_char_p),
        "hot_abi_version": ([], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    if path == LIB_PATH:
        _lib = lib
    return lib


def check(lib, rc: int) -> None:
    if rc != HOT_OK:
        raise HotError(rc, lib.hot_last_error().decode())
