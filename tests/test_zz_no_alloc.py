"""The allocation-free GSW entry point through the C ABI against hot_gsw (needs an MI355X).

hot_gsw_noalloc runs the same kernels with every buffer in the library's fixed per-GPU workspace,
so its results must equal hot_gsw's bit for bit; two calls in a row, the second smaller than the
first, check that what a call leaves in the workspace does not leak into the next one.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.parity import assert_phase, assert_V, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu case] {request.node.nodeid}", file=sys.stderr, flush=True)
    yield


def same(a, b):
    assert torch.equal(a.phase, b.phase)
    assert torch.equal(a.V, b.V)
    np.testing.assert_array_equal(a.stats, b.stats)
    if a.w is not None:
        assert torch.equal(a.w, b.w) and torch.equal(a.theta, b.theta)


def test_no_alloc_equals_hot_gsw_twice_shrinking(hot):
    cases = [(W.c2(), 50), (W.random_problem(612, 300, 77, 37), 6)]  # the second call is smaller
    with hot.Context(0) as c:
        for p, K in cases:
            ref = c.hot_gsw(p.slm, p.xyz, p.theta0, K, state=True)
            got = c.hot_gsw_noalloc(p.slm, p.xyz, p.theta0, K, state=True)
            torch.cuda.synchronize()
            same(got, ref)
        # the smaller problem against the oracle as well (the bar of the parity tests)
        p, K = cases[1]
        o = oracle.solve("gsw", p.slm, p.xyz, p.theta0, K)
        assert_phase(to_np(got.phase), o["phi"])
        assert_V(to_np(got.V), o["V"])


def test_no_alloc_seeded_and_warm_started(hot):
    """Trap phases from the seed, then a warm start from the exported weights and phases."""
    p = W.random_problem(613, 200, 120, 24)
    with hot.Context(0) as c:
        ref = c.hot_gsw(p.slm, p.xyz, None, 4, seed=77, state=True)
        got = c.hot_gsw_noalloc(p.slm, p.xyz, None, 4, seed=77, state=True)
        torch.cuda.synchronize()
        same(got, ref)
        th = to_np(ref.theta)
        ref2 = c.hot_gsw(p.slm, p.xyz, th, 3, w0=ref.w.clone(), state=True)
        got2 = c.hot_gsw_noalloc(p.slm, p.xyz, th, 3, w0=got.w.clone(), state=True)
        torch.cuda.synchronize()
        same(got2, ref2)


def test_no_alloc_rejects_what_does_not_fit(hot):
    """2048 traps leave room for about 43000 iterations of statistics; more is refused before any
    device work, and the next call still works."""
    p = W.Problem(W.Slm(64, 64), W.square_grid(46, 3e-6)[:2048], W.random_phases(614, 2048), 0)
    with hot.Context(0) as c:
        with pytest.raises(hot.HotError) as e:
            c.hot_gsw_noalloc(p.slm, p.xyz, p.theta0, 50000, stats=False)
        assert e.value.code == hot.HOT_EINVAL
        q = W.random_problem(615, 96, 64, 9)
        ref = c.hot_gsw(q.slm, q.xyz, q.theta0, 3)
        got = c.hot_gsw_noalloc(q.slm, q.xyz, q.theta0, 3)
        torch.cuda.synchronize()
        same(got, ref)
