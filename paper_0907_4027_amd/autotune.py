"""Autotuner for the launch-shape knobs of the C ABI (``hot_set_tuning``).

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
