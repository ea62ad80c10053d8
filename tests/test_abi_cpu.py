"""C-ABI contract on the CPU: the library loads, exports every symbol include/hot.h
declares, rejects bad arguments on the host before any device work, and reports
HOT_EDEVICE when no GPU is present.  No compute calls are made here."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_0907_4027_amd import _lib
from tests.conftest import gpu_available

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "hot.h")


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hot_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(_lib.EXPORTS)


def test_header_constants_match_binding():
    """Every enum and #define constant the header gives (error codes, variants, tuning keys, limits)
    has the same value in the binding."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    consts = {k: int(v) for k, v in re.findall(r"\b(HOT_[A-Z0-9_]+)\s*=\s*(-?\d+)", text)}
    consts.update({k: int(v) for k, v in re.findall(r"#define\s+(HOT_[A-Z0-9_]+)\s+(-?\d+)", text)})
    assert len(consts) >= 15
    for name, value in consts.items():
        if name == "HOT_ABI_VERSION":
            continue
        assert hasattr(_lib, name), name
        assert getattr(_lib, name) == value, (name, getattr(_lib, name), value)


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_abi_version(lib):
    assert lib.hot_abi_version() == 1


def test_struct_layouts():
    assert C.sizeof(_lib.hot_slm) == 32
    assert C.sizeof(_lib.hot_stats) == 12


def slm(nx=64, ny=48, pitch=15e-6, lam=1.064e-6, f=5e-3):
    return _lib.hot_slm(nx, ny, pitch, lam, f)


def xyz_ptr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


@pytest.mark.parametrize("case,expect", [
    ("ok", _lib.HOT_OK),
    ("nx0", _lib.HOT_EINVAL), ("ny_big", _lib.HOT_EINVAL), ("pitch_neg", _lib.HOT_EINVAL),
    ("lam_nan", _lib.HOT_EINVAL), ("focal_inf", _lib.HOT_EINVAL), ("m0", _lib.HOT_EINVAL),
    ("m_big", _lib.HOT_EINVAL), ("xyz_nan", _lib.HOT_EINVAL), ("xyz_null", _lib.HOT_EINVAL),
    ("iters_neg", _lib.HOT_EINVAL), ("slm_null", _lib.HOT_EINVAL),
])
def test_check_problem(lib, case, expect):
    s = slm()
    M, iters = 5, 3
    a = np.zeros((max(M, 1), 3))
    if case == "nx0":
        s.nx = 0
    elif case == "ny_big":
        s.ny = _lib.HOT_MAX_SIDE + 1
    elif case == "pitch_neg":
        s.pitch = -1e-6
    elif case == "lam_nan":
        s.wavelength = math.nan
    elif case == "focal_inf":
        s.focal = math.inf
    elif case == "m0":
        M = 0
    elif case == "m_big":
        M = _lib.HOT_MAX_TRAPS + 1
        a = np.zeros((M, 3))
    elif case == "xyz_nan":
        a[2, 1] = math.nan
    elif case == "iters_neg":
        iters = -1
    a, p = xyz_ptr(a)
    if case == "xyz_null":
        p = None
    sp = None if case == "slm_null" else C.byref(s)
    rc = lib.hot_check_problem(sp, M, p, iters)
    assert rc == expect
    if expect != _lib.HOT_OK:
        assert len(lib.hot_last_error()) > 0


@pytest.mark.skipif(gpu_available(), reason="checks the GPU-less error path")
def test_create_without_gpu_reports_edevice(lib):
    ctx = C.c_void_p()
    assert lib.hot_create(C.byref(ctx), 0, None) == _lib.HOT_EDEVICE
    assert ctx.value is None
    assert b"device" in lib.hot_last_error()


def test_null_context_is_rejected_before_any_device_work(lib):
    s = slm()
    a, p = xyz_ptr(np.zeros((3, 3)))
    cnt = (C.c_int32 * 1)(3)
    assert lib.hot_rs(None, C.byref(s), 3, p, None, 0, None, None, None) == _lib.HOT_EINVAL
    assert lib.hot_gs(None, C.byref(s), 3, p, None, 0, 2, None, None, None) == _lib.HOT_EINVAL
    assert lib.hot_gsw(None, C.byref(s), 3, p, None, 0, 2, None, None, None, None, None, None) == _lib.HOT_EINVAL
    assert lib.hot_gsw_batched(None, C.byref(s), 1, cnt, p, p, 2, None, None, None) == _lib.HOT_EINVAL
    assert lib.hot_forward_V(None, C.byref(s), 1, cnt, p, None, None) == _lib.HOT_EINVAL
    assert lib.hot_adjoint(None, C.byref(s), 1, cnt, p, None, None, None) == _lib.HOT_EINVAL
    assert lib.hot_set_variant(None, 0) == _lib.HOT_EINVAL
    assert lib.hot_sync(None) == _lib.HOT_EINVAL
    assert lib.hot_destroy(None) == _lib.HOT_OK
    assert b"ctx" in lib.hot_last_error()


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(ImportError):
        _lib.load(str(tmp_path / "nope.so"))
