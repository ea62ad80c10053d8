"""The HIP path at the shapes of the benchmarked workloads, through the C ABI (needs an MI355X).

* 64 holograms of 512^2 with 4..256 traps each, 30 GSW iterations, in one batched call: eight of
  them, spanning the trap counts, against the oracle run on each alone.
* 8 x 512^2 x 64 traps, Eq. 1 and its adjoint in one batched call each, and through the
  autograd Function with the trap-intensity loss, against the oracle per hologram; uneven trap
  counts on a ragged grid; the Adam loop against an FP64 Adam driven by the oracle's gradient.
* The stored-matrix variant at the benchmarked sizes (512^2 x 100 and 1024^2 x 256).
* Identical-input checks of single passes: the oracle is handed the GPU's own weights and trap
  phases (pixel pass, Eq. 3) or the GPU's own phase mask (trap pass, Eq. 1) after every iteration,
  so the comparison measures one pass of FP32 arithmetic, not the GSW map's amplification of it.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.parity import as_complex, assert_phase, assert_stats, assert_V, to_np, wrapped_diff

pytestmark = pytest.mark.gpu

VARIANTS = ["onthefly", "separable"]


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu case] {request.node.nodeid}", file=sys.stderr, flush=True)
    yield


@pytest.fixture(scope="module", params=VARIANTS)
def vctx(hot, request):
    c = hot.Context(0)
    c.set_variant(request.param)
    yield c
    c.close()


_CACHE = {}


def cached(key, fn):
    if key not in _CACHE:
        _CACHE[key] = fn()
    return _CACHE[key]


# ------------------------------------------------------------------ 64 holograms, 30 iterations

# indices of the workload's holograms at the 0th, 1/8, ..., 7/8 and last place of their sorted
# trap counts (19, 54, 96, 128, 149, 172, 224 and 252 traps)
C4_PICK = (22, 58, 54, 51, 34, 45, 17, 29)


def test_batched_64_holograms_30_iterations_match_oracle(vctx):
    bt = W.c4()
    assert bt.b == 64 and bt.iters == 30
    r = vctx.hot_gsw_batched(bt.slm, bt.counts, bt.xyz, bt.theta0, bt.iters)
    torch.cuda.synchronize()
    ph, V, st = to_np(r.phase), to_np(r.V), r.stats
    o = bt.offsets()
    ms = sorted(int(bt.counts[b]) for b in C4_PICK)
    assert ms[0] == int(bt.counts.min()) and ms[-1] == int(bt.counts.max())
    for b in C4_PICK:
        p = bt.problem(b)
        ref = cached(("c4", b), lambda: oracle.solve("gsw", p.slm, p.xyz, p.theta0, bt.iters))
        assert_phase(ph[b], ref["phi"], what=f"hologram {b} (M={p.m})")
        assert_V(V[o[b]:o[b + 1]], ref["V"], what=f"hologram {b} (M={p.m})")
        assert_stats(st[b], ref["stats"])


# ------------------------------------------------------------------ 8 x 512^2 x 64: Eq. 1 and its adjoint

def c5_inputs():
    """The 8-hologram workload with each hologram's random-superposition mask (the starting point
    of its Adam loop), rounded to FP32, and a random complex G per trap."""
    def make():
        bt = W.c5()
        o = bt.offsets()
        phis = np.stack([oracle.backward(bt.slm, bt.xyz[o[b]:o[b + 1]], None, bt.theta0[o[b]:o[b + 1]])
                         for b in range(bt.b)]).astype(np.float32).astype(np.float64)
        rng = np.random.default_rng(505)
        G = (rng.normal(size=int(bt.counts.sum())) + 1j * rng.normal(size=int(bt.counts.sum())))
        return bt, phis, G.astype(np.complex64).astype(np.complex128)
    return cached("c5", make)


def to_dev(phis, slm):
    return torch.tensor(phis.reshape(-1, slm.ny, slm.nx), dtype=torch.float32, device="cuda")


def test_batched_forward_V_8x512sq_64(vctx):
    bt, phis, _ = c5_inputs()
    V = to_np(vctx.hot_forward_V(bt.slm, bt.counts, bt.xyz, to_dev(phis, bt.slm)))
    torch.cuda.synchronize()
    o = bt.offsets()
    for b in range(bt.b):
        ref = cached(("c5V", b), lambda: oracle.forward(bt.slm, bt.xyz[o[b]:o[b + 1]], phis[b]))
        assert_V(V[o[b]:o[b + 1]], ref, what=f"hologram {b}")
        np.testing.assert_allclose(as_complex(V[o[b]:o[b + 1]]), ref, atol=2e-6)


def test_batched_adjoint_8x512sq_64(vctx):
    bt, phis, G = c5_inputs()
    Gt = torch.tensor(np.stack([G.real, G.imag], -1), dtype=torch.float32, device="cuda")
    g = to_np(vctx.hot_adjoint(bt.slm, bt.counts, bt.xyz, to_dev(phis, bt.slm), Gt)).reshape(bt.b, -1)
    torch.cuda.synchronize()
    o = bt.offsets()
    for b in range(bt.b):
        ref = cached(("c5adj", b), lambda: oracle.adjoint(bt.slm, bt.xyz[o[b]:o[b + 1]], phis[b], G[o[b]:o[b + 1]]))
        rel = np.linalg.norm(g[b] - ref) / np.linalg.norm(ref)
        assert rel <= 1e-4, (b, rel)


def test_trap_field_gradient_8x512sq_64(hot, vctx):
    """The autograd Function over the whole batch: the summed trap-intensity loss and, per hologram,
    its gradient (the other holograms' terms do not depend on this hologram's mask) against the
    oracle's loss and analytic gradient."""
    bt, phis, _ = c5_inputs()
    phase = to_dev(phis, bt.slm).requires_grad_(True)
    V = hot.TrapField.apply(phase, vctx, bt.slm, bt.counts, bt.xyz)
    L = hot.trap_intensity_loss(V, bt.counts)
    L.backward()
    g = to_np(phase.grad).reshape(bt.b, -1)
    o = bt.offsets()
    Ltot = 0.0
    for b in range(bt.b):
        Lo, Vo, go = cached(("c5lg", b), lambda: oracle.loss_grad(bt.slm, bt.xyz[o[b]:o[b + 1]], phis[b]))
        Ltot += Lo
        rel = np.linalg.norm(g[b] - go) / np.linalg.norm(go)
        assert rel <= 1e-4, (b, rel)
    assert abs(L.item() - Ltot) <= 1e-4 * abs(Ltot)


@pytest.mark.parametrize("turns", [300, 3000])
def test_unwrapped_caller_phase(vctx, turns):
    """A caller's mask need not lie in [0, 2 pi): a GS mask plus 2 pi k per pixel, |k| up to `turns`
    (far past the 256 revolutions of the hardware sin/cos), gives Eq. 1 and its adjoint of the same
    FP32 values within the usual bars."""
    p = W.random_problem(540, 300, 77, 64)
    phi0 = to_np(vctx.hot_gs(p.slm, p.xyz, p.theta0, 5).phase).ravel()
    rng = np.random.default_rng(541)
    k = rng.integers(-turns, turns + 1, p.slm.n)
    phi = (phi0 + 2 * math.pi * k).astype(np.float32).astype(np.float64)
    assert np.abs(phi).max() > 2 * math.pi * 0.9 * turns
    G = (rng.normal(size=p.m) + 1j * rng.normal(size=p.m)).astype(np.complex64).astype(np.complex128)
    Gt = torch.tensor(np.stack([G.real, G.imag], -1), dtype=torch.float32, device="cuda")
    ph = to_dev(phi[None], p.slm)
    V = to_np(vctx.hot_forward_V(p.slm, [p.m], p.xyz, ph))
    g = to_np(vctx.hot_adjoint(p.slm, [p.m], p.xyz, ph, Gt)).ravel()
    torch.cuda.synchronize()
    assert_V(V, oracle.forward(p.slm, p.xyz, phi))
    ref = oracle.adjoint(p.slm, p.xyz, phi, G)
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    assert rel <= 1e-4, rel


@pytest.mark.parametrize("counts", [(3, 64, 131, 17), (1, 200)])
def test_batched_adjoint_uneven_counts(vctx, counts):
    """Uneven trap counts on a grid ragged in both directions: every hologram's Eq. 1 and gradient."""
    slm = W.Slm(300, 77)
    probs = [W.random_problem(520 + i, slm.nx, slm.ny, m) for i, m in enumerate(counts)]
    xyz = np.concatenate([p.xyz for p in probs])
    rng = np.random.default_rng(530)
    phis = rng.uniform(0, 2 * math.pi, (len(counts), slm.n)).astype(np.float32).astype(np.float64)
    G = (rng.normal(size=sum(counts)) + 1j * rng.normal(size=sum(counts))).astype(np.complex64).astype(np.complex128)
    Gt = torch.tensor(np.stack([G.real, G.imag], -1), dtype=torch.float32, device="cuda")
    ph = to_dev(phis, slm)
    V = to_np(vctx.hot_forward_V(slm, list(counts), xyz, ph))
    g = to_np(vctx.hot_adjoint(slm, list(counts), xyz, ph, Gt)).reshape(len(counts), -1)
    torch.cuda.synchronize()
    o = 0
    for b, p in enumerate(probs):
        assert_V(V[o:o + p.m], oracle.forward(slm, p.xyz, phis[b]), what=f"hologram {b}")
        ref = oracle.adjoint(slm, p.xyz, phis[b], G[o:o + p.m])
        rel = np.linalg.norm(g[b] - ref) / np.linalg.norm(ref)
        assert rel <= 1e-4, (b, rel)
        o += p.m


def adam_fp64(slm, xyz, phi0, steps, lr=0.05, b1=0.9, b2=0.999, eps=1e-8):
    """Adam with torch's default constants on the oracle's loss and analytic gradient, in FP64."""
    phi = phi0.copy()
    m = np.zeros_like(phi)
    v = np.zeros_like(phi)
    losses = []
    for t in range(1, steps + 1):
        L, _, g = oracle.loss_grad(slm, xyz, phi)
        losses.append(L)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        phi = phi - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return phi, np.array(losses)


def test_adam_loop_matches_fp64_adam(hot, vctx):
    """Five Adam steps (lr 0.05) on the 64^2, 4-trap case from its random-superposition mask: the
    loss at every step and the final mask against the same loop in FP64 on the oracle's gradient;
    then the full 200-step loop lowers the loss."""
    p, _ = W.c5_fd_case()
    phi0 = oracle.backward(p.slm, p.xyz, None, p.theta0).astype(np.float32).astype(np.float64)
    ph0 = to_dev(phi0, p.slm)
    phase, losses = hot.optimize_phase(vctx, p.slm, [p.m], p.xyz, ph0, steps=5, lr=0.05)
    ref_phi, ref_losses = adam_fp64(p.slm, p.xyz, phi0, 5)
    np.testing.assert_allclose(losses.cpu().numpy(), ref_losses, rtol=1e-4)
    assert_phase(to_np(phase).ravel(), ref_phi, what="mask after 5 Adam steps")
    _, long = hot.optimize_phase(vctx, p.slm, [p.m], p.xyz, ph0, steps=200, lr=0.05)
    long = long.cpu().numpy()
    assert np.all(np.isfinite(long))
    assert long[-1] < long[0] and long[-10:].max() < long[:10].min(), (long[0], long[-1])


def test_adam_loop_8x512sq_64_lowers_the_loss(hot, vctx):
    """The workload's own Adam loop (8 x 512^2, 64 traps each, lr 0.05) from the random-superposition
    masks: the first step's loss matches the oracle's and the loss falls over 200 steps."""
    bt, phis, _ = c5_inputs()
    phase, losses = hot.optimize_phase(vctx, bt.slm, bt.counts, bt.xyz, to_dev(phis, bt.slm), steps=200, lr=0.05)
    losses = losses.cpu().numpy()
    o = bt.offsets()
    L0 = sum(cached(("c5lg", b), lambda: oracle.loss_grad(bt.slm, bt.xyz[o[b]:o[b + 1]], phis[b]))[0]
             for b in range(bt.b))
    assert abs(losses[0] - L0) <= 1e-4 * abs(L0)
    assert np.all(np.isfinite(losses)) and losses[-1] < losses[0]


# ------------------------------------------------------------------ identical-input single passes

def per_pass_check(ctx, p, ks, idx=None, frac=0.999):
    """After k = 0, 1, ... GSW iterations: the pixel pass (the returned mask) against the oracle's
    Eq. 3 on the GPU's own weights and trap phases, and the trap pass (the returned V) against the
    oracle's Eq. 1 on the GPU's own mask."""
    for k in ks:
        g = ctx.hot_gsw(p.slm, p.xyz, p.theta0, k, state=True)
        torch.cuda.synchronize()
        phi = to_np(g.phase).ravel()
        w, th = to_np(g.w), to_np(g.theta)
        ref = oracle.backward(p.slm, p.xyz, w, th, idx=idx)
        assert_phase(phi if idx is None else phi[idx], ref, frac=frac, what=f"pixel pass after {k} iterations")
        assert_V(to_np(g.V), oracle.forward(p.slm, p.xyz, phi), what=f"trap pass after {k} iterations")


def test_odd_grid_130_traps_every_iteration(vctx):
    """129 x 65 pixels, 130 traps (many phase vortices): each of the 7 masks of a 6-iteration GSW
    run and its V, each pass on identical inputs, at the parity bar."""
    p = W.random_problem(205, 129, 65, 130)
    per_pass_check(vctx, p, range(7))


def test_1024sq_256_traps_final_passes(vctx):
    """The 1024^2 x 256 workload after its 40 iterations: the final pixel pass on 65536 sampled
    pixels and the final trap pass in full, on identical inputs, at the parity bar."""
    p = W.c3()
    idx = np.random.default_rng(8).choice(p.slm.n, 65536, replace=False)
    per_pass_check(vctx, p, [p.iters], idx=idx)


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_stored_variant_at_benchmark_sizes(hot, name):
    """The stored-matrix variant in the configurations the benchmark times it in: 512^2 x 100 after
    50 iterations (a 210 MB matrix) and 1024^2 x 256 after 40 (2.15 GB): the final pixel pass (in
    full, or on 65536 sampled pixels at 1024^2) and the final trap pass, on identical inputs, at
    the parity bar."""
    p = getattr(W, name)()
    idx = None if name == "c2" else np.random.default_rng(9).choice(p.slm.n, 65536, replace=False)
    with hot.Context(0) as c:
        c.set_variant("stored")
        per_pass_check(c, p, [p.iters], idx=idx)
