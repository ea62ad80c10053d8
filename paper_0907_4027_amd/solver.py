"""Python face of the C ABI: a `Context` whose methods share the ABI's names.

Only marshalling happens here -- torch tensors provide device memory and the
stream; every step of every solver runs in the HIP kernels behind libhot.so.
"""
from __future__ import annotations

import ctypes as C
from typing import NamedTuple, Optional

import numpy as np
import torch

from . import _lib
from ._lib import HOT_ONTHEFLY, HOT_SEPARABLE, HOT_STORED, check, hot_slm, hot_stats


class Result(NamedTuple):
    phase: torch.Tensor                 # [ny, nx] (or [B, ny, nx]) float32 radians
    V: torch.Tensor                     # [M, 2] (or [sum M, 2]) float32 (re, im)
    stats: Optional[np.ndarray]         # [K+1, 3] (or [B, K+1, 3]): efficiency, uniformity, sigma
    w: Optional[torch.Tensor] = None    # [M] final weights (GSW)
    theta: Optional[torch.Tensor] = None  # [M] final trap phases (GSW)


def as_slm(slm) -> hot_slm:
    if isinstance(slm, hot_slm):
        return slm
    if isinstance(slm, dict):
        return hot_slm(int(slm["nx"]), int(slm["ny"]), float(slm["pitch"]), float(slm["wavelength"]),
                       float(slm["focal"]))
    return hot_slm(int(slm.nx), int(slm.ny), float(slm.pitch), float(slm.wavelength), float(slm.focal))


def _host_f64(a, rows: Optional[int] = None, cols: Optional[int] = None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if cols is not None and (a.ndim != 2 or a.shape[1] != cols):
        raise ValueError(f"expected an array of shape [n, {cols}], got {a.shape}")
    if rows is not None and a.shape[0] != rows:
        raise ValueError(f"expected {rows} rows, got {a.shape[0]}")
    return a


def _dp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _vp(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """A hot_ctx bound to one GPU and (by default) torch's current stream on it."""

    def __init__(self, device: int = 0, stream=None):
        self._lib = _lib.load()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        elif isinstance(stream, torch.cuda.Stream):
            stream = stream.cuda_stream
        ptr = C.c_void_p()
        check(self._lib, self._lib.hot_create(C.byref(ptr), device, C.c_void_p(stream)))
        self._ctx = ptr

    # -- lifetime -------------------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_ctx", None):
            self._lib.hot_destroy(self._ctx)
            self._ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- configuration --------------------------------------------------------------
    def set_variant(self, variant) -> None:
        v = {"onthefly": HOT_ONTHEFLY, "stored": HOT_STORED, "separable": HOT_SEPARABLE}.get(variant, variant)
        check(self._lib, self._lib.hot_set_variant(self._ctx, int(v)))

    def set_tuning(self, pixels_per_lane: int = 0, traps_per_lane: int = 0, segment: int = 0,
                   slices: int = 0, sep_waves: int = 0, sep_chunk: int = 0, rows: int = 0,
                   sep_split: int = 0, fract: int = 0) -> None:
        """Launch-shape knobs (0 = built-in choice); see hot_set_tuning in include/hot.h."""
        for key, val in ((_lib.HOT_TUNE_PIXELS_PER_LANE, pixels_per_lane), (_lib.HOT_TUNE_TRAPS_PER_LANE, traps_per_lane),
                         (_lib.HOT_TUNE_SEGMENT, segment), (_lib.HOT_TUNE_SLICES, slices),
                         (_lib.HOT_TUNE_SEP_WAVES, sep_waves), (_lib.HOT_TUNE_SEP_CHUNK, sep_chunk),
                         (_lib.HOT_TUNE_ROWS, rows), (_lib.HOT_TUNE_SEP_SPLIT, sep_split),
                         (_lib.HOT_TUNE_FRACT, fract)):
            check(self._lib, self._lib.hot_set_tuning(self._ctx, key, int(val)))

    def set_graphs(self, enabled: bool) -> None:
        """Replay captured hipGraphs of repeated solves (default) or launch eagerly."""
        check(self._lib, self._lib.hot_set_tuning(self._ctx, _lib.HOT_TUNE_GRAPHS, int(bool(enabled))))

    def set_stream(self, stream=None) -> None:
        if isinstance(stream, torch.cuda.Stream):
            stream = stream.cuda_stream
        check(self._lib, self._lib.hot_set_stream(self._ctx, C.c_void_p(stream)))

    def hot_sync(self) -> None:
        check(self._lib, self._lib.hot_sync(self._ctx))

    # -- helpers --------------------------------------------------------------------
    def _dev(self, t: Optional[torch.Tensor], numel: int, name: str) -> Optional[torch.Tensor]:
        if t is None:
            return None
        if not (t.is_cuda and t.device == self.device and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float32 tensor on {self.device}")
        if t.numel() != numel:
            raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
        return t

    def _new(self, *shape) -> torch.Tensor:
        return torch.empty(*shape, dtype=torch.float32, device=self.device)

    # -- single hologram -------------------------------------------------------------
    def hot_rs(self, slm, xyz, theta0=None, seed: int = 0, phase=None, V=None, stats: bool = True) -> Result:
        s = as_slm(slm)
        x = _host_f64(xyz, cols=3)
        M = x.shape[0]
        th = None if theta0 is None else _host_f64(theta0, rows=M)
        phase = self._dev(phase, s.nx * s.ny, "phase") if phase is not None else self._new(s.ny, s.nx)
        V = self._dev(V, 2 * M, "V") if V is not None else self._new(M, 2)
        st = (hot_stats * 1)() if stats else None
        check(self._lib, self._lib.hot_rs(self._ctx, C.byref(s), M, _dp(x), _dp(th), C.c_uint64(seed), _vp(phase),
                                          _vp(V), st))
        return Result(phase, V, _stats_np(st, (1, 3)))

    def hot_gs(self, slm, xyz, theta0=None, iters: int = 10, seed: int = 0, phase=None, V=None,
               stats: bool = True) -> Result:
        s = as_slm(slm)
        x = _host_f64(xyz, cols=3)
        M = x.shape[0]
        th = None if theta0 is None else _host_f64(theta0, rows=M)
        phase = self._dev(phase, s.nx * s.ny, "phase") if phase is not None else self._new(s.ny, s.nx)
        V = self._dev(V, 2 * M, "V") if V is not None else self._new(M, 2)
        st = (hot_stats * (iters + 1))() if stats else None
        check(self._lib, self._lib.hot_gs(self._ctx, C.byref(s), M, _dp(x), _dp(th), C.c_uint64(seed), int(iters),
                                          _vp(phase), _vp(V), st))
        return Result(phase, V, _stats_np(st, (iters + 1, 3)))

    def hot_gsw(self, slm, xyz, theta0=None, iters: int = 10, seed: int = 0, w0=None, phase=None, V=None,
                stats: bool = True, state: bool = False, w_out=None, theta_out=None) -> Result:
        """GSW; with state=True the final weights and trap phases are returned (written into
        w_out / theta_out when given, e.g. to reuse buffers frame after frame)."""
        s = as_slm(slm)
        x = _host_f64(xyz, cols=3)
        M = x.shape[0]
        th = None if theta0 is None else _host_f64(theta0, rows=M)
        w0 = self._dev(w0, M, "w0")
        phase = self._dev(phase, s.nx * s.ny, "phase") if phase is not None else self._new(s.ny, s.nx)
        V = self._dev(V, 2 * M, "V") if V is not None else self._new(M, 2)
        w_out = self._dev(w_out, M, "w_out") if w_out is not None else (self._new(M) if state else None)
        th_out = self._dev(theta_out, M, "theta_out") if theta_out is not None else (self._new(M) if state else None)
        st = (hot_stats * (iters + 1))() if stats else None
        check(self._lib, self._lib.hot_gsw(self._ctx, C.byref(s), M, _dp(x), _dp(th), C.c_uint64(seed), int(iters),
                                           _vp(w0), _vp(w_out), _vp(th_out), _vp(phase), _vp(V), st))
        return Result(phase, V, _stats_np(st, (iters + 1, 3)), w_out, th_out)

    def hot_gsw_noalloc(self, slm, xyz, theta0=None, iters: int = 10, seed: int = 0, w0=None, phase=None, V=None,
                        stats: bool = True, state: bool = False, w_out=None, theta_out=None) -> Result:
        """GSW through the allocation-free entry point (the library's fixed per-GPU workspace);
        arguments and results as hot_gsw.  Output tensors are allocated here by torch when not given."""
        s = as_slm(slm)
        x = _host_f64(xyz, cols=3)
        M = x.shape[0]
        th = None if theta0 is None else _host_f64(theta0, rows=M)
        w0 = self._dev(w0, M, "w0")
        phase = self._dev(phase, s.nx * s.ny, "phase") if phase is not None else self._new(s.ny, s.nx)
        V = self._dev(V, 2 * M, "V") if V is not None else self._new(M, 2)
        w_out = self._dev(w_out, M, "w_out") if w_out is not None else (self._new(M) if state else None)
        th_out = self._dev(theta_out, M, "theta_out") if theta_out is not None else (self._new(M) if state else None)
        st = (hot_stats * (iters + 1))() if stats else None
        check(self._lib, self._lib.hot_gsw_noalloc(self._ctx, C.byref(s), M, _dp(x), _dp(th), C.c_uint64(seed),
                                                   int(iters), _vp(w0), _vp(w_out), _vp(th_out), _vp(phase), _vp(V),
                                                   st))
        return Result(phase, V, _stats_np(st, (iters + 1, 3)), w_out, th_out)

    # -- batches ---------------------------------------------------------------------
    def hot_gsw_batched(self, slm, counts, xyz, theta0, iters: int = 10, phase=None, V=None,
                        stats: bool = True) -> Result:
        s = as_slm(slm)
        cnt = np.ascontiguousarray(counts, dtype=np.int32)
        B, T = cnt.shape[0], int(cnt.sum())
        x = _host_f64(xyz, rows=T, cols=3)
        th = _host_f64(theta0, rows=T)
        phase = self._dev(phase, B * s.nx * s.ny, "phase") if phase is not None else self._new(B, s.ny, s.nx)
        V = self._dev(V, 2 * T, "V") if V is not None else self._new(T, 2)
        st = (hot_stats * (B * (iters + 1)))() if stats else None
        check(self._lib, self._lib.hot_gsw_batched(self._ctx, C.byref(s), B, cnt.ctypes.data_as(C.POINTER(C.c_int32)),
                                                   _dp(x), _dp(th), int(iters), _vp(phase), _vp(V), st))
        return Result(phase, V, _stats_np(st, (B, iters + 1, 3)))

    def hot_forward_V(self, slm, counts, xyz, phase: torch.Tensor, V=None) -> torch.Tensor:
        s = as_slm(slm)
        cnt = np.ascontiguousarray(counts, dtype=np.int32)
        B, T = cnt.shape[0], int(cnt.sum())
        x = _host_f64(xyz, rows=T, cols=3)
        self._dev(phase, B * s.nx * s.ny, "phase")
        V = self._dev(V, 2 * T, "V") if V is not None else self._new(T, 2)
        check(self._lib, self._lib.hot_forward_V(self._ctx, C.byref(s), B, cnt.ctypes.data_as(C.POINTER(C.c_int32)),
                                                 _dp(x), _vp(phase), _vp(V)))
        return V

    def hot_encode_u8(self, phase: torch.Tensor, frame: Optional[torch.Tensor] = None) -> torch.Tensor:
        """8-bit SLM frame of a phase mask: rint(phase * 256 / 2 pi) mod 256 (device uint8)."""
        if not (phase.is_cuda and phase.device == self.device and phase.dtype == torch.float32
                and phase.is_contiguous()):
            raise ValueError(f"phase must be a contiguous float32 tensor on {self.device}")
        if frame is None:
            frame = torch.empty(phase.shape, dtype=torch.uint8, device=self.device)
        elif not (frame.dtype == torch.uint8 and frame.is_contiguous() and frame.numel() == phase.numel()
                  and frame.device == self.device):
            raise ValueError("frame must be a contiguous uint8 tensor with as many elements as phase")
        check(self._lib, self._lib.hot_encode_u8(self._ctx, phase.numel(), _vp(phase), _vp(frame)))
        return frame

    def hot_time_passes(self, slm, xyz, theta0, reps: int = 20) -> np.ndarray:
        """Mean device ms per launch, back to back, of [iteration kernel, reduction into V, pixel pass
        alone, trap pass alone] (the reduction runs once per solve on the on-the-fly path)."""
        s = as_slm(slm)
        x = _host_f64(xyz, cols=3)
        M = x.shape[0]
        th = _host_f64(theta0, rows=M)
        phase, V = self._new(s.ny, s.nx), self._new(M, 2)
        ms = (C.c_float * 4)()
        check(self._lib, self._lib.hot_time_passes(self._ctx, C.byref(s), M, _dp(x), _dp(th), int(reps),
                                                   _vp(phase), _vp(V), ms))
        return np.array(ms[:], dtype=np.float64)

    def hot_pixel_pass_variant(self, slm, xyz, theta0, placement: str = "lds", mapping: str = "linear",
                               block: int = 256, reps: int = 20, phase=None):
        """Random-superposition pixel pass with the trap records in LDS / read by scalar loads / read by
        per-lane global loads, pixels in row segments or square tiles (the ablation of the paper's
        Table 1).  Returns (phase [ny, nx], mean ms per launch)."""
        s = as_slm(slm)
        x = _host_f64(xyz, cols=3)
        M = x.shape[0]
        th = _host_f64(theta0, rows=M)
        pl = {"lds": _lib.HOT_REC_LDS, "scalar": _lib.HOT_REC_SCALAR, "global": _lib.HOT_REC_GLOBAL}[placement]
        mp = {"linear": _lib.HOT_MAP_LINEAR, "square": _lib.HOT_MAP_SQUARE}[mapping]
        phase = self._dev(phase, s.nx * s.ny, "phase") if phase is not None else self._new(s.ny, s.nx)
        ms = (C.c_float * 1)()
        check(self._lib, self._lib.hot_pixel_pass_variant(self._ctx, C.byref(s), M, _dp(x), _dp(th), int(pl), int(mp),
                                                          int(block), int(reps), _vp(phase), ms))
        return phase, float(ms[0])

    def hot_probe_issue(self, kind: int, waves_per_simd: int, reps: int) -> dict:
        """Issue-rate micro-benchmark (kind 0 FMA, 1 sin/cos, 2 the direct passes' term); see
        include/hot.h.  Returns rates per second, the waves' mean shader clock and timings."""
        out = (C.c_double * 6)()
        check(self._lib, self._lib.hot_probe_issue(self._ctx, int(kind), int(waves_per_simd), int(reps), out))
        return {"ops_per_s": out[0], "clock_hz": out[1], "span_s": out[2], "event_s": out[3],
                "cycles_per_wave": out[4], "waves": int(out[5])}

    def hot_probe_copy(self, src: torch.Tensor, dst: torch.Tensor, reps: int = 20) -> dict:
        """Device copy bandwidth (bytes read + written per second) with the library's copy kernel."""
        if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()
                and src.numel() * src.element_size() == dst.numel() * dst.element_size()):
            raise ValueError("src and dst must be contiguous device tensors of the same byte size")
        out = (C.c_double * 2)()
        nbytes = src.numel() * src.element_size()
        check(self._lib, self._lib.hot_probe_copy(self._ctx, _vp(src), _vp(dst), int(nbytes), int(reps), out))
        return {"bytes_per_s": out[0], "ms_per_copy": out[1]}

    def hot_adjoint(self, slm, counts, xyz, phase: torch.Tensor, G: torch.Tensor, grad=None) -> torch.Tensor:
        s = as_slm(slm)
        cnt = np.ascontiguousarray(counts, dtype=np.int32)
        B, T = cnt.shape[0], int(cnt.sum())
        x = _host_f64(xyz, rows=T, cols=3)
        self._dev(phase, B * s.nx * s.ny, "phase")
        self._dev(G, 2 * T, "G")
        grad = self._dev(grad, B * s.nx * s.ny, "grad") if grad is not None else self._new(*phase.shape)
        check(self._lib, self._lib.hot_adjoint(self._ctx, C.byref(s), B, cnt.ctypes.data_as(C.POINTER(C.c_int32)),
                                               _dp(x), _vp(phase), _vp(G), _vp(grad)))
        return grad


def _stats_np(st, shape):
    if st is None:
        return None
    a = np.ctypeslib.as_array(C.cast(st, C.POINTER(C.c_float)), shape=(int(np.prod(shape)),))
    return a.reshape(shape).astype(np.float64)
