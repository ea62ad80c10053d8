"""Real-time frame loop of the paper's interactive demonstration (Section 5).

Per frame: the traps move (the caller passes their new positions), a few GSW
iterations run warm-started from the previous frame's weights and trap phases,
the phase mask is encoded as the 8-bit SLM frame (grey level linear in phase
over 0..2 pi), and the frame is copied into pinned host memory, where a display
path would pick it up.  All device work goes through the C ABI; buffers are
fixed, so every frame after the first replays the same captured graph.
"""
from __future__ import annotations

import time

import numpy as np
import torch


class RealtimeLoop:
    def __init__(self, ctx, slm, m: int, iters: int = 5):
        self.ctx, self.slm, self.m, self.iters = ctx, slm, int(m), int(iters)
        dev = ctx.device
        self.phase = torch.empty(slm.ny, slm.nx, device=dev)
        self.V = torch.empty(self.m, 2, device=dev)
        self.w = torch.ones(self.m, device=dev)
        self.theta_dev = torch.empty(self.m, device=dev)
        self.frame_dev = torch.empty(slm.ny, slm.nx, dtype=torch.uint8, device=dev)
        self.frame_host = torch.empty(slm.ny, slm.nx, dtype=torch.uint8, pin_memory=True)
        self.theta_host = torch.empty(self.m, dtype=torch.float32, pin_memory=True)
        self.V_host = torch.empty(self.m, 2, dtype=torch.float32, pin_memory=True)
        self.theta = None
        self.started = False

    def frame(self, xyz, theta0=None):
        """Compute and deliver one frame; returns (frame [ny, nx] uint8 host tensor, V host
        tensor [M, 2], seconds from call to frame in host memory)."""
        t0 = time.perf_counter()
        if not self.started:
            th = np.asarray(theta0, dtype=np.float64)
            w0 = None
        else:
            th = self.theta
            w0 = self.w
        self.ctx.hot_gsw(self.slm, xyz, th, self.iters, w0=w0, phase=self.phase, V=self.V, stats=False,
                         state=True, w_out=self.w, theta_out=self.theta_dev)
        self.ctx.hot_encode_u8(self.phase, self.frame_dev)
        self.frame_host.copy_(self.frame_dev, non_blocking=True)
        self.theta_host.copy_(self.theta_dev, non_blocking=True)
        self.V_host.copy_(self.V, non_blocking=True)
        torch.cuda.current_stream(self.ctx.device).synchronize()
        self.theta = self.theta_host.numpy().astype(np.float64)
        self.started = True
        return self.frame_host, self.V_host, time.perf_counter() - t0
