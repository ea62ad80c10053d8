"""Differentiable trap fields: Eq. 1 forward and its adjoint behind torch.autograd.

`TrapField.apply(phase, ctx, slm, counts, xyz)` returns V ([sum M, 2], re/im) for the
phase masks `phase` ([B, ny, nx]); its backward calls the hand-written adjoint kernel
(hot_adjoint), which recomputes the propagation phases Delta instead of storing them.
"""
from __future__ import annotations

import torch


class TrapField(torch.autograd.Function):
    @staticmethod
    def forward(fctx, phase, hctx, slm, counts, xyz):
        phase = phase.contiguous()
        V = hctx.hot_forward_V(slm, counts, xyz, phase)
        fctx.save_for_backward(phase)
        fctx.hctx, fctx.args = hctx, (slm, counts, xyz)
        return V

    @staticmethod
    def backward(fctx, gV):
        (phase,) = fctx.saved_tensors
        slm, counts, xyz = fctx.args
        # G_m = dL/dRe V_m + i dL/dIm V_m is exactly gV laid out as interleaved (re, im)
        grad = fctx.hctx.hot_adjoint(slm, counts, xyz, phase, gV.contiguous().to(torch.float32))
        return grad, None, None, None, None


def trap_intensity_loss(V: torch.Tensor, counts) -> torch.Tensor:
    """Sum over holograms of  -sum_m log I_m + 10 var(I)/mean(I)^2  (population variance),
    I_m = |V_m|^2: high efficiency (log term) and uniformity (variance term)."""
    I = (V.double() ** 2).sum(-1)
    total = I.new_zeros(())
    o = 0
    for m in [int(c) for c in counts]:
        Ib = I[o:o + m]
        mu = Ib.mean()
        total = total - torch.log(Ib).sum() + 10.0 * Ib.var(unbiased=False) / mu ** 2
        o += m
    return total


def optimize_phase(hctx, slm, counts, xyz, phase0: torch.Tensor, steps: int = 200, lr: float = 0.05):
    """Adam (torch defaults, lr 0.05) on the trap-intensity loss; returns (phase, losses)."""
    phase = phase0.clone().requires_grad_(True)
    opt = torch.optim.Adam([phase], lr=lr)
    losses = []
    for _ in range(steps):
        opt.zero_grad(set_to_none=True)
        V = TrapField.apply(phase, hctx, slm, counts, xyz)
        loss = trap_intensity_loss(V, counts)
        loss.backward()
        opt.step()
        losses.append(loss.detach())
    return phase.detach(), torch.stack(losses)
