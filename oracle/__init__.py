"""FP64 CPU oracle of the hologram solver -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product (``paper_0907_4027_amd``)
never does, and this package never imports the product: the two share no code.

The arithmetic lives in ``oracle.c`` (plain C99, libm, double precision, OpenMP
over pixels); this module only builds it with gcc and marshals numpy arrays.
Each wrapper names the passage of the paper it follows (see oracle.c).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

RS, GS, GSW = 0, 1, 2
_ALGO = {"rs": RS, "gs": GS, "gsw": GSW}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, IEEE double: no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def configure(lib):
    """Declare the C signatures on a loaded oracle library (also used for planted-mistake builds)."""
    d, i, i64 = C.c_double, C.c_int, C.c_int64
    P = C.c_void_p
    lib.orc_backward.argtypes = [i, i, d, d, d, i, P, P, P, i64, P, P, P]
    lib.orc_backward.restype = None
    lib.orc_forward.argtypes = [i, i, d, d, d, i, P, P, P]
    lib.orc_forward.restype = i
    lib.orc_stats.argtypes = [i, P, P]
    lib.orc_stats.restype = None
    lib.orc_theta_seed.argtypes = [i, C.c_uint64, P]
    lib.orc_theta_seed.restype = None
    lib.orc_solve.argtypes = [i, i, i, d, d, d, i, P, P, P, i, P, P, P, P, P, P, P]
    lib.orc_solve.restype = i
    lib.orc_adjoint.argtypes = [i, i, d, d, d, i, P, P, P, P]
    lib.orc_adjoint.restype = None
    lib.orc_loss_grad.argtypes = [i, i, d, d, d, i, P, P, P, P]
    lib.orc_loss_grad.restype = d
    lib.orc_set_threads.argtypes = [i]
    lib.orc_set_threads.restype = i
    lib.orc_get_threads.argtypes = []
    lib.orc_get_threads.restype = i
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = configure(C.CDLL(_LIB))
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _geo(slm):
    return int(slm.nx), int(slm.ny), float(slm.pitch), float(slm.wavelength), float(slm.focal)


def set_threads(n: int) -> int:
    return _load().orc_set_threads(int(n))


def get_threads() -> int:
    return _load().orc_get_threads()


def backward(slm, xyz, w, theta, idx=None, return_field=False):
    """Eq. 3 with weights: phi_j = arg sum_m w_m exp(i(Delta_j^m + theta_m)) in [0, 2 pi)."""
    xyz, theta = _f64(xyz), _f64(theta)
    w = None if w is None else _f64(w)
    n = int(slm.nx) * int(slm.ny) if idx is None else len(idx)
    idx_a = None if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
    phi = np.empty(n)
    S = np.empty(2 * n) if return_field else None
    _load().orc_backward(*_geo(slm), xyz.shape[0], _p(xyz), _p(w), _p(theta), n, _p(idx_a), _p(phi), _p(S))
    if return_field:
        return phi, S[0::2] + 1j * S[1::2]
    return phi


def forward(slm, xyz, phi) -> np.ndarray:
    """Eq. 1: V_m = (1/N) sum_j exp(i(phi_j - Delta_j^m)); returns complex [M]."""
    xyz, phi = _f64(xyz), _f64(phi).ravel()
    assert phi.size == int(slm.nx) * int(slm.ny)
    V = np.empty(2 * xyz.shape[0])
    rc = _load().orc_forward(*_geo(slm), xyz.shape[0], _p(xyz), _p(phi), _p(V))
    if rc:
        raise RuntimeError(f"orc_forward failed ({rc})")
    return V[0::2] + 1j * V[1::2]


def stats(V) -> np.ndarray:
    """Section 3 efficiency e, uniformity u, and sigma = std(I)/mean(I)."""
    v = np.empty(2 * len(V))
    v[0::2], v[1::2] = np.real(V), np.imag(V)
    out = np.empty(3)
    _load().orc_stats(len(V), _p(v), _p(out))
    return out


def theta_seed(m: int, seed: int) -> np.ndarray:
    """SplitMix64-derived trap phases, used when no theta0 is supplied."""
    out = np.empty(m)
    _load().orc_theta_seed(m, C.c_uint64(seed), _p(out))
    return out


def solve(algo, slm, xyz, theta0, iters: int = 0, w0=None, trace: bool = False) -> dict:
    """RS / GS / GSW.  Returns dict(phi, V, stats[(K+1),3], w, theta[, w_trace, V_trace])."""
    a = _ALGO[algo] if isinstance(algo, str) else int(algo)
    xyz, theta0 = _f64(xyz), _f64(theta0)
    M = xyz.shape[0]
    K = 0 if a == RS else int(iters)
    N = int(slm.nx) * int(slm.ny)
    phi, V = np.empty(N), np.empty(2 * M)
    st = np.empty(3 * (K + 1))
    w_out, th_out = np.empty(M), np.empty(M)
    w0a = None if w0 is None else _f64(w0)
    wt = np.empty((K + 1) * M) if trace else None
    vt = np.empty((K + 1) * 2 * M) if trace else None
    rc = _load().orc_solve(a, *_geo(slm), M, _p(xyz), _p(theta0), _p(w0a), K, _p(phi), _p(V), _p(st),
                           _p(w_out), _p(th_out), _p(wt), _p(vt))
    if rc:
        raise RuntimeError(f"orc_solve failed ({rc})")
    out = dict(phi=phi, V=V[0::2] + 1j * V[1::2], stats=st.reshape(K + 1, 3), w=w_out, theta=th_out)
    if trace:
        out["w_trace"] = wt.reshape(K + 1, M)
        vt = vt.reshape(K + 1, M, 2)
        out["V_trace"] = vt[..., 0] + 1j * vt[..., 1]
    return out


def adjoint(slm, xyz, phi, G) -> np.ndarray:
    """dL/dphi_j = (1/N) Im(exp(-i phi_j) sum_m G_m exp(i Delta_j^m)) for G_m = dL/dReV + i dL/dImV."""
    xyz, phi = _f64(xyz), _f64(phi).ravel()
    g = np.empty(2 * len(G))
    g[0::2], g[1::2] = np.real(G), np.imag(G)
    out = np.empty(phi.size)
    _load().orc_adjoint(*_geo(slm), xyz.shape[0], _p(xyz), _p(phi), _p(g), _p(out))
    return out


def loss_grad(slm, xyz, phi, with_grad: bool = True):
    """L = -sum log I_m + 10 var(I)/mean(I)^2 and its analytic gradient over phi."""
    xyz, phi = _f64(xyz), _f64(phi).ravel()
    V = np.empty(2 * xyz.shape[0])
    grad = np.empty(phi.size) if with_grad else None
    L = _load().orc_loss_grad(*_geo(slm), xyz.shape[0], _p(xyz), _p(phi), _p(V), _p(grad))
    return L, V[0::2] + 1j * V[1::2], grad
