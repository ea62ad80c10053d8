"""Autotuner for the launch-shape knobs of the C ABI (``hot_set_tuning``).

Two entry points: ``tune``/``sweep`` for one hologram (back-to-back launches of the fused
iteration kernel through ``hot_time_passes``) and ``tune_batched``/``sweep_batched`` for a batch of
holograms with uneven trap counts (short batched solves timed with HIP events on the context's
stream).

For one problem shape it times every candidate combination of

    pixels_per_lane  (pixel pass: 1 or 2 pixels per lane, i.e. 512- or 256-thread rows on 512-wide rows)
    segment          (pixels of a row per block: the whole row, 256 or 512)
    traps_per_lane   (trap pass: traps each lane accumulates; 0 = the library's cycle model)
    rows             (rows per block, 1 or 2: two rows share one update and one set of trap sums)

with ``hot_time_passes`` (HIP events around back-to-back launches on the context's stream),
keeps the fastest fused-iteration kernel, and caches it in a JSON file keyed by
(architecture, variant, grid, trap-count bucket).  The sweep table doubles as an
ablation of the kernel's shape choices on this GPU.  Only launch shapes change --
results differ at most by FP32 summation order.
"""
from __future__ import annotations

import itertools
import json
import os
from typing import Optional

import torch

from .solver import Context

CANDIDATES = {
    "pixels_per_lane": (1, 2),
    "segment": (0, 256, 512),
    "traps_per_lane": (0, 2, 3, 4, 5, 6, 8),
    "rows": (1, 2),
}
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "hot_mi355x", "tuning.json")


def _bucket(m: int) -> int:
    b = 1
    while b < m:
        b *= 2
    return b


def cache_key(ctx: Context, slm, m: int, variant: str = "onthefly") -> str:
    arch = torch.cuda.get_device_properties(ctx.device).gcnArchName.split(":")[0]
    return f"{arch}/{variant}/{int(slm.nx)}x{int(slm.ny)}/M{_bucket(m)}"


def sweep(ctx: Context, slm, xyz, theta0, reps: int = 20, candidates: Optional[dict] = None) -> list:
    """Time every knob combination; returns rows sorted by the fused-iteration time."""
    cand = candidates or CANDIDATES
    rows = []
    for q, seg, tpl, nr in itertools.product(cand["pixels_per_lane"], cand["segment"], cand["traps_per_lane"],
                                             cand.get("rows", (1,))):
        if seg == 256 and q == 2:
            continue  # same launch as (q=1, seg=256)
        if nr == 2 and q == 1 and seg != 256 and int(slm.nx) > 256:
            continue  # 512-thread rows: two rows per block are not built
        ctx.set_tuning(pixels_per_lane=q, segment=seg, traps_per_lane=tpl, rows=nr)
        ms = ctx.hot_time_passes(slm, xyz, theta0, reps=reps)
        rows.append({"pixels_per_lane": q, "segment": seg, "traps_per_lane": tpl, "rows": nr,
                     "iteration_us": round(float(ms[0]) * 1e3, 3), "reduce_us": round(float(ms[1]) * 1e3, 3),
                     "pixel_pass_us": round(float(ms[2]) * 1e3, 3), "trap_pass_us": round(float(ms[3]) * 1e3, 3)})
    ctx.set_tuning()
    rows.sort(key=lambda r: r["iteration_us"])
    return rows


def tune(ctx: Context, slm, xyz, theta0, cache: Optional[str] = DEFAULT_CACHE, reps: int = 20,
         apply: bool = True) -> dict:
    """Best knobs for this problem shape (from the cache, or measured and cached); applied to
    ctx when `apply`.  Returns {"key", "knobs", "table" (None on a cache hit)}."""
    key = cache_key(ctx, slm, len(xyz))
    db = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            db = json.load(f)
    table = None
    if key not in db:
        table = sweep(ctx, slm, xyz, theta0, reps=reps)
        best = table[0]
        db[key] = {k: best[k] for k in ("pixels_per_lane", "segment", "traps_per_lane", "rows")} | \
                  {"iteration_us": best["iteration_us"]}
        if cache:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(db, f, indent=1, sort_keys=True)
    knobs = {k: db[key][k] for k in ("pixels_per_lane", "segment", "traps_per_lane", "rows") if k in db[key]}
    if apply:
        ctx.set_tuning(**knobs)
    return {"key": key, "knobs": knobs, "table": table}


BATCH_CANDIDATES = {
    "traps_per_lane": (0, 2, 3, 4, 5, 6, 8),
    "rows": (1, 2),
    "pixels_per_lane": (0, 1),
}


def batch_key(ctx: Context, slm, counts, variant: str = "onthefly") -> str:
    """Cache key of a batch: architecture, grid, batch size and the trap-count distribution
    (quartiles bucketed to powers of two)."""
    arch = torch.cuda.get_device_properties(ctx.device).gcnArchName.split(":")[0]
    import numpy as np
    q = [_bucket(int(v)) for v in np.quantile(np.asarray(counts), (0.0, 0.25, 0.5, 0.75, 1.0))]
    return f"{arch}/{variant}/batched/{int(slm.nx)}x{int(slm.ny)}/B{len(counts)}/M" + "-".join(map(str, q))


def sweep_batched(ctx: Context, slm, counts, xyz, theta0, iters: int = 2, reps: int = 3,
                  candidates: Optional[dict] = None) -> list:
    """Time hot_gsw_batched (a short solve of `iters` iterations, graph-replayed) for every knob
    combination; rows sorted by device milliseconds per solve."""
    import numpy as np
    cand = candidates or BATCH_CANDIDATES
    cnt = np.asarray(counts, dtype=np.int32)
    B, T = len(cnt), int(cnt.sum())
    phase = torch.empty(B, int(slm.ny), int(slm.nx), device=ctx.device)
    V = torch.empty(T, 2, device=ctx.device)
    rows = []
    for tpl, nr, q in itertools.product(cand["traps_per_lane"], cand["rows"], cand["pixels_per_lane"]):
        try:
            ctx.set_tuning(traps_per_lane=tpl, rows=nr, pixels_per_lane=q)
            run = lambda: ctx.hot_gsw_batched(slm, cnt, xyz, theta0, iters, phase=phase, V=V, stats=False)
            run()
            torch.cuda.synchronize(ctx.device)
        except Exception:  # a shape the library refuses for this batch (e.g. two rows on 512-thread rows)
            continue
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        torch.cuda.synchronize(ctx.device)
        rows.append({"traps_per_lane": tpl, "rows": nr, "pixels_per_lane": q,
                     "ms_per_solve": round(e0.elapsed_time(e1) / reps, 4)})
    ctx.set_tuning()
    rows.sort(key=lambda r: r["ms_per_solve"])
    return rows


def tune_batched(ctx: Context, slm, counts, xyz, theta0, cache: Optional[str] = DEFAULT_CACHE, iters: int = 2,
                 reps: int = 3, apply: bool = True) -> dict:
    """Best knobs for this batch shape (cached like ``tune``); applied to ctx when `apply`."""
    key = batch_key(ctx, slm, counts)
    db = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            db = json.load(f)
    table = None
    if key not in db:
        table = sweep_batched(ctx, slm, counts, xyz, theta0, iters=iters, reps=reps)
        best = table[0]
        db[key] = {k: best[k] for k in ("traps_per_lane", "rows", "pixels_per_lane")} | \
                  {"ms_per_solve": best["ms_per_solve"]}
        if cache:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(db, f, indent=1, sort_keys=True)
    knobs = {k: db[key][k] for k in ("traps_per_lane", "rows", "pixels_per_lane")}
    if apply:
        ctx.set_tuning(**knobs)
    return {"key": key, "knobs": knobs, "table": table}


TABLE1_VARIANTS = [(pl, mp, bs) for pl in ("lds", "scalar", "global") for mp in ("linear", "square") for bs in (64, 256)]


def table1_sweep(ctx: Context, slm, xyz, theta0, reps: int = 20) -> list:
    """The MI355X analogue of the paper's Table 1 (Section 4): the random-superposition pixel pass
    with the trap records in LDS, read by scalar loads or read by every lane from global memory,
    pixels in row segments or square tiles, blocks of 64 or 256 pixels; rows sorted by time, with
    the paper's unit (ms per trap) and terms per second."""
    n, m = int(slm.nx) * int(slm.ny), len(xyz)
    rows = []
    for pl, mp, bs in TABLE1_VARIANTS:
        _, ms = ctx.hot_pixel_pass_variant(slm, xyz, theta0, placement=pl, mapping=mp, block=bs, reps=reps)
        rows.append({"placement": pl, "mapping": mp, "block": bs, "ms_per_pass": round(ms, 5),
                     "ms_per_trap": round(ms / m, 6), "terms_per_s": n * m / (ms * 1e-3)})
    rows.sort(key=lambda r: r["ms_per_pass"])
    return rows
