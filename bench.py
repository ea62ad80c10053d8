#!/usr/bin/env python3
"""Benchmark of the MI355X hologram solver (one JSON line on stdout).

Step = one weighted Gerchberg-Saxton solve (Section 3 / Fig. 2 of Bianchi & Di
Leonardo, arXiv:0907.4027) of the 512 x 512 SLM, 100 random 3D traps, 50
iterations workload, called through the C ABI with its inputs already resident
(trap tables cached on the device, phase/V buffers preallocated).

    value = N * M * K / t   pixel-trap updates per second (one update = one (pixel, trap)
                            pair in one iteration = one term in each of the two passes)

Also reported: the pass timings behind the roofline object (HIP events on the
library's stream), the batched (64 holograms) and adjoint (8 x forward + adjoint)
modes against plain per-hologram launches, the stored-exp(i Delta) variant, and
the FP64 CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs at the published 2.4 GHz.  The minimum work of a (pixel, trap) term of
# either direct pass is 2 FMA for the phase, sin + cos, 2 FMA to accumulate.  Issue model: a wave64
# FMA takes 4 shader cycles of its SIMD and a sin or cos 8, with no overlap: 32 cycles per wave of
# 64 terms, 4.915e12 terms/s.  The probe of exactly that instruction mix (hot_probe_issue kind 2,
# profiles/peaks_mi355x.md) runs faster than the model at high occupancy: 30.86 cycles per wave of
# terms at 8 waves per SIMD.  The roofline takes that measured best as the peak (the stricter of the
# two), scaled to the published clock.
SIMDS = 256 * 4
MODEL_CYCLES_PER_WAVE_TERM = 32.0
PROBED_CYCLES_PER_WAVE_TERM = 30.86
MODEL_TERMS_PER_S = SIMDS * 2.4e9 * 64 / MODEL_CYCLES_PER_WAVE_TERM
PEAK_TERMS_PER_S = SIMDS * 2.4e9 * 64 / PROBED_CYCLES_PER_WAVE_TERM
HBM_PEAK_GBS = 8000.0
MFMA_F32_PEAK_TFLOPS = 157.3  # dense FP32 matrix-core peak of the MI355X
K_SHORT = 0  # iterations of the shorter solve (the RS pass alone) whose time difference gives the per-launch duration


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None once the kernel
    source has changed since the counters were taken (the summary records its SHA-256)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic_gsw-512sq-100traps.md")
    src = os.path.join(ROOT, "paper_0907_4027_amd", "csrc", "hot_kernels.hip")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"kernel source sha256: ([0-9a-f]{64})", text)
    m_b = re.search(r"HBM bytes per launch: ([0-9.eE+]+)", text)
    if not m_sha or not m_b:
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m_sha.group(1):
        return None
    return float(m_b.group(1))


def time_calls(fn, reps, sync):
    import torch
    sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    sync()
    return e0.elapsed_time(e1) / reps


def time_wall(fn, reps, sync):
    """Mean wall-clock ms per call of fn over reps calls, the device synchronised before and after."""
    sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    sync()
    return (time.perf_counter() - t0) / reps * 1e3


def measure_peaks(ctx, log):
    """Issue rates of the FP32 vector pipes (FMA, sin/cos, and the direct passes' term mix) at 1, 2,
    4 and 8 waves per SIMD with the shader clock each ran at, and the device copy bandwidth, all
    from the library's probe kernels.  The roofline's peak assumes 2.4 GHz, one FMA per SIMD per 4
    cycles and sin/cos at half that rate with no overlap (8 issue slots per term); the 'model' ratios
    below compare each measured rate with that model at the measured clock."""
    import torch
    # shader cycles per lane operation in the model: a wave64 FMA takes 4, a sin or cos 8, a term
    # (4 FMA + sin + cos) 32
    # The matrix kinds count FLOPs, against the published FP32 matrix peak (157.3 TFLOP/s at
    # 2.4 GHz: 64 FLOPs per SIMD per cycle, a 16x16x4 product every 32 cycles)
    kinds = {0: ("fma", 4.0 / 64), 1: ("sincos", 8.0 / 64), 2: ("term", 32.0 / 64),
             3: ("mfma_16x16x4_f32", 1.0 / 64), 4: ("mfma_16x16x4_f32_one_accumulator", 1.0 / 64),
             5: ("mfma_32x32x2_f32", 1.0 / 64), 6: ("mfma_16x16x4_f32_with_sincos", 1.0 / 64)}
    res = {}
    simds = 256 * 4
    for kind, (name, cyc_per_op) in kinds.items():
        rows = {}
        for wps in (1, 2, 4, 8):
            reps = 40000 // wps
            r = ctx.hot_probe_issue(kind, wps, reps)
            model = simds * r["clock_hz"] / cyc_per_op   # lane operations per second per the model
            model_24 = simds * 2.4e9 / cyc_per_op
            rows[str(wps)] = {"ops_per_s": r["ops_per_s"], "clock_GHz": round(r["clock_hz"] / 1e9, 4),
                              "vs_model_at_measured_clock": round(r["ops_per_s"] / model, 4),
                              "vs_model_at_2.4GHz": round(r["ops_per_s"] / model_24, 4),
                              "span_ms": round(r["span_s"] * 1e3, 3), "event_ms": round(r["event_s"] * 1e3, 3)}
        res[name] = rows
        if kind >= 3:
            for v in rows.values():
                v["cycles_per_product_per_SIMD"] = round((4096 if kind == 5 else 2048) * SIMDS * v["clock_GHz"] * 1e9
                                                         / v["ops_per_s"], 2)
        log(f"[bench] probe {name}: " + "  ".join(
            f"{w}w {v['ops_per_s'] / 1e12:.2f}T/s @{v['clock_GHz']:.2f}GHz ({v['vs_model_at_measured_clock']:.3f})"
            for w, v in rows.items()))
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, device="cuda")
    dst = torch.empty_like(src)
    cp = ctx.hot_probe_copy(src, dst, reps=20)
    del src, dst
    res["copy"] = {"bytes": nbytes, "GBs_read_plus_write": round(cp["bytes_per_s"] / 1e9, 1),
                   "ms_per_copy": round(cp["ms_per_copy"], 4), "frac_of_8TBs": round(cp["bytes_per_s"] / 8e12, 4)}
    log(f"[bench] probe copy 1 GiB: {cp['bytes_per_s'] / 1e9:.0f} GB/s read+write")
    best = max(v["ops_per_s"] / (SIMDS * v["clock_GHz"] * 1e9) for v in res["term"].values())  # terms per SIMD cycle
    res["model"] = {"fma_cycles_per_wave_instruction": 4, "sincos_cycles_per_wave_instruction": 8,
                    "term_cycles_per_wave": MODEL_CYCLES_PER_WAVE_TERM,
                    "model_terms_per_s_at_2.4GHz": MODEL_TERMS_PER_S,
                    "term_cycles_per_wave_measured_best": round(64.0 / best, 3),
                    "peak_terms_per_s_used": PEAK_TERMS_PER_S,
                    "peak_cycles_per_wave_term_used": PROBED_CYCLES_PER_WAVE_TERM}
    return res


def onthefly_line(ctx, q, log, reps=10):
    """One single-hologram GSW workload on the default (on-the-fly) kernels: time per solve from
    graph replays, the iteration kernel's in-situ duration (slope against a zero-iteration solve),
    updates/s, its fraction of the term roofline, and the figures of merit of every iteration."""
    import torch
    sync = torch.cuda.synchronize
    ph = torch.empty(q.slm.ny, q.slm.nx, device="cuda")
    Vq = torch.empty(q.m, 2, device="cuda")

    def solve(k):
        return lambda: ctx.hot_gsw(q.slm, q.xyz, q.theta0, k, phase=ph, V=Vq, stats=False)
    solve(q.iters)()
    solve(0)()
    t = time_calls(solve(q.iters), reps, sync)
    t0 = time_calls(solve(0), reps, sync)
    per = (t - t0) / q.iters
    terms = 2.0 * q.slm.n * q.m
    st = ctx.hot_gsw(q.slm, q.xyz, q.theta0, q.iters, phase=ph, V=Vq, stats=True).stats
    log(f"[bench] {q.name} on-the-fly: {t:.4f} ms per solve, iteration {per * 1e3:.2f} us in situ, "
        f"final e={st[-1, 0]:.4f} u={st[-1, 1]:.4f} sigma={st[-1, 2]:.4f}")
    return {"nx": q.slm.nx, "ny": q.slm.ny, "traps": q.m, "iterations": q.iters, "ms_per_solve": round(t, 4),
            "updates_per_s": q.slm.n * q.m * q.iters / (t * 1e-3), "holograms_per_s": 1e3 / t,
            "iteration_in_situ_us": round(per * 1e3, 3),
            "frac_of_term_roofline": round(terms / (per * 1e-3) / PEAK_TERMS_PER_S, 4),
            "per_iteration": {"efficiency": [round(float(v), 5) for v in st[:, 0]],
                              "uniformity": [round(float(v), 5) for v in st[:, 1]],
                              "sigma": [round(float(v), 5) for v in st[:, 2]]}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip batched / adjoint / stored comparisons")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner's launch-shape sweep")
    ap.add_argument("--only", choices=["main", "passes", "tune", "batched", "adjoint", "stored", "interactive", "separable",
                                       "fig7", "counters", "peaks", "workloads"], default=None,
                    help="run one section only (for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X; sharding a batch or one "
              "hologram's rows over several GPUs is not built (pass --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_0907_4027_amd as hot
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    ctx = hot.Context(0)
    sync = torch.cuda.synchronize
    out = {}

    # ---------------------------------------------------------------- headline: GSW 512^2 x 100, 50 iterations
    p = W.c2()
    N, M, K = p.slm.n, p.m, p.iters
    phase = torch.empty(p.slm.ny, p.slm.nx, device="cuda")
    V = torch.empty(M, 2, device="cuda")

    def step():
        main_ctx.hot_gsw(p.slm, p.xyz, p.theta0, K, phase=phase, V=V, stats=False)

    ms = None
    in_situ_ms = None
    end_to_end_ms = None
    tuning = None
    main_ctx = ctx  # the headline runs the library's own launch shape
    if args.only in (None, "tune") and not args.no_tune:
        # ablation: the autotuner's sweep of the launch-shape knobs on its own context; the headline
        # keeps the library's choice so that profiles and counters describe the same kernel
        from paper_0907_4027_amd import autotune
        with hot.Context(0) as tctx:
            tr = autotune.tune(tctx, p.slm, p.xyz, p.theta0, cache=None, reps=20, apply=False)
            pd = tctx.hot_time_passes(p.slm, p.xyz, p.theta0, reps=20)
            # the paper's Table 1 axes on its SR grid (768 x 768), 100 traps in the workloads' box
            t1slm = W.Slm(768, 768)
            t1 = autotune.table1_sweep(tctx, t1slm, p.xyz, p.theta0, reps=20)
        table = tr["table"]
        default = {"iteration_us": round(float(pd[0]) * 1e3, 3), "reduce_us": round(float(pd[1]) * 1e3, 3)}
        tuning = {"best_knobs": tr["knobs"], "best": table[0], "library_default": default, "worst": table[-1],
                  "configurations": len(table),
                  "best_vs_default": round(default["iteration_us"] / table[0]["iteration_us"], 4),
                  "table1": {"workload": "random-superposition pixel pass, 768 x 768 SLM, 100 traps (the paper's "
                                         "Table 1 axes: record placement, pixel mapping, block size)",
                             "rows": t1,
                             "paper_context": "GTX 260, 768^2: 0.35 ms per trap with all rules, 1.22 without shared-"
                                              "memory records (other hardware)"}}
        log("[bench] table 1 axes: " + "  ".join(f"{r['placement']}/{r['mapping']}/{r['block']}: {r['ms_per_pass'] * 1e3:.1f}us"
                                                  for r in t1))
        log(f"[bench] autotune sweep: best {tr['knobs']} {table[0]['iteration_us']} us, library default "
            f"{default['iteration_us']} us, worst {table[-1]['iteration_us']} us over {len(table)} shapes")
    if args.only in (None, "main"):
        for _ in range(args.warmup):
            step()
        sync()
        t0 = time.perf_counter()
        ms = time_calls(step, args.steps, sync)
        wall = time.perf_counter() - t0
        log(f"[bench] gsw {p.name}: {ms:.4f} ms/step ({args.steps} steps, wall {wall:.3f} s)")
        # the iteration kernel's duration inside the solve: one launch per iteration, so the slope of
        # the solve time over the iteration count (same problem, K_SHORT iterations) is its average
        # launch duration, launch gaps included
        def step_short():
            main_ctx.hot_gsw(p.slm, p.xyz, p.theta0, K_SHORT, phase=phase, V=V, stats=False)
        for _ in range(args.warmup):
            step_short()
        ms_short = time_calls(step_short, args.steps, sync)
        in_situ_ms = (ms - ms_short) / (K - K_SHORT)
        log(f"[bench] {K_SHORT}-iteration solve {ms_short:.4f} ms: iteration kernel in situ {in_situ_ms * 1e3:.2f} us")
        # correctness of what was timed: final stats from one more synchronising call
        st = main_ctx.hot_gsw(p.slm, p.xyz, p.theta0, K, phase=phase, V=V, stats=True).stats
        log(f"[bench] final e={st[-1, 0]:.4f} u={st[-1, 1]:.4f} sigma={st[-1, 2]:.4f}")
        # end to end from the host: trap geometry in, the solve with its statistics (one stream
        # synchronisation), the phase mask and V copied to pinned host memory
        h_phase = torch.empty(phase.shape, dtype=phase.dtype, pin_memory=True)
        h_V = torch.empty(V.shape, dtype=V.dtype, pin_memory=True)

        def e2e():
            main_ctx.hot_gsw(p.slm, p.xyz, p.theta0, K, phase=phase, V=V, stats=True)
            h_phase.copy_(phase)
            h_V.copy_(V)
        e2e()
        sync()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            e2e()
        end_to_end_ms = (time.perf_counter() - t0) / args.steps * 1e3
        log(f"[bench] end to end (host geometry in, stats sync, phase + V to pinned host) {end_to_end_ms:.4f} ms")

    # ---------------------------------------------------------------- hardware-counter runs
    if args.only == "counters":
        # a plain device-to-device copy of known size (FETCH_SIZE / WRITE_SIZE calibration), then a few
        # launches of every kernel family: the headline iteration kernel (in the per-pass timing below),
        # the stored variant's passes at 512^2 x 100 and 1024^2 x 256, and the separable iteration
        src = torch.ones(64 << 20, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        sync()
        del src, dst
        log("[bench] counters: 3 copies of 256 MiB")
        for variant, probs, reps in (("stored", (W.c2(), W.c3()), 3), ("separable", (W.c2(), W.c3()), 5)):
            with hot.Context(0) as cc:
                cc.set_variant(variant)
                for q in probs:
                    pm = cc.hot_time_passes(q.slm, q.xyz, q.theta0, reps=reps)
                    log(f"[bench] counters: {variant} {q.name} passes {pm[0]:.4f} {pm[2]:.4f} {pm[3]:.4f} ms")
        sync()

    # ---------------------------------------------------------------- per-pass timings -> roofline
    roof = None
    if args.only in (None, "main", "passes", "counters"):
        pm = main_ctx.hot_time_passes(p.slm, p.xyz, p.theta0, reps=50)
        terms = N * M
        log(f"[bench] ms/launch back to back: iteration kernel {pm[0]:.4f}  collect {pm[1]:.4f}  "
            f"pixel pass alone {pm[2]:.4f}  trap pass alone {pm[3]:.4f}")
        # dominant kernel: the fused iteration kernel, 2 terms (one per pass) per (pixel, trap), over
        # its average duration inside the timed solves (else, without them, back to back)
        dur_ms = in_situ_ms if in_situ_ms is not None else float(pm[0])
        achieved = 2 * terms / (dur_ms * 1e-3) / 1e9
        peak = PEAK_TERMS_PER_S / 1e9
        roof = {"bound": "alu", "kernel": "k_iter (GSW update + pixel pass + trap pass + trap sums, fused)",
                "achieved": round(achieved, 1), "peak": round(peak, 1), "unit": "Gterm/s",
                "frac": round(achieved / peak, 4), "frac_vs_issue_model": round(achieved * 1e9 / MODEL_TERMS_PER_S, 4),
                "peak_basis": "term-mix probe's best, 30.86 shader cycles per wave of 64 terms, at 2.4 GHz x 1024 SIMDs",
                "traffic": measured_traffic("k_iter"),
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "duration": "in situ (solve-time slope over iterations)" if in_situ_ms is not None
                            else "back-to-back launches",
                "ms_per_launch": {"iteration_in_situ": None if in_situ_ms is None else round(in_situ_ms, 5),
                                  "iteration_back_to_back": round(float(pm[0]), 5),
                                  "collect_once_per_solve": round(float(pm[1]), 5),
                                  "pixel_pass_alone": round(float(pm[2]), 5), "trap_pass_alone": round(float(pm[3]), 5)},
                "frac_pixel_pass_alone": round(terms / (pm[2] * 1e-3) / PEAK_TERMS_PER_S, 4),
                "frac_trap_pass_alone": round(terms / (pm[3] * 1e-3) / PEAK_TERMS_PER_S, 4)}

    # ---------------------------------------------------------------- the other single-hologram workloads, on-the-fly
    if not args.no_extra and args.only in (None, "workloads"):
        out["workloads"] = {q.name: onthefly_line(ctx, q, log) for q in (W.c1(), W.c3())}

    # ---------------------------------------------------------------- batched: 64 holograms vs 64 plain launches
    if not args.no_extra and args.only in (None, "batched"):
        from paper_0907_4027_amd import autotune
        bt = W.c4()
        T = int(bt.counts.sum())
        bph = torch.empty(bt.b, bt.slm.ny, bt.slm.nx, device="cuda")
        bV = torch.empty(T, 2, device="cuda")
        o = bt.offsets()
        bctx = hot.Context(0)  # the batched launch with the autotuner's shape for this batch
        tb_res = autotune.tune_batched(bctx, bt.slm, bt.counts, bt.xyz, bt.theta0, cache=None)

        def batched():
            bctx.hot_gsw_batched(bt.slm, bt.counts, bt.xyz, bt.theta0, bt.iters, phase=bph, V=bV, stats=False)

        def sequential():
            for b in range(bt.b):
                ctx.hot_gsw(bt.slm, bt.xyz[o[b]:o[b + 1]], bt.theta0[o[b]:o[b + 1]], bt.iters,
                            phase=bph[b], V=bV[o[b]:o[b + 1]], stats=False)

        batched()
        sequential()  # every hologram's captured graph is now cached (one per output buffer)
        sync()
        tb = time_calls(batched, 3, sync)
        ts = time_calls(sequential, 2, sync)
        tbw = time_wall(batched, 3, sync)
        tsw = time_wall(sequential, 2, sync)
        upd = bt.slm.n * T * bt.iters
        # whole batched solve (31 launches of the fused kernel plus the per-solve kernels) against
        # the issue-slot roofline: 2 terms per pixel-trap update, plus the initial pass
        terms = 2.0 * bt.slm.n * T * (bt.iters + 1)
        table = tb_res["table"]
        out["batched"] = {"workload": f"{bt.name}: 64 x 512^2, M in [4,256] (sum {T}), 30 iterations",
                          "ms": round(tb, 3), "updates_per_s": upd / (tb * 1e-3), "holograms_per_s": bt.b / (tb * 1e-3),
                          "plain_ms": round(ts, 3), "plain_updates_per_s": upd / (ts * 1e-3),
                          "speedup_vs_plain": round(ts / tb, 3),
                          "timing": "device: HIP events on the stream around the calls; wall: host clock with a final "
                                    "synchronisation; the plain form replays each hologram's cached graph",
                          "wall_ms": round(tbw, 3), "plain_wall_ms": round(tsw, 3),
                          "autotuned_shape": tb_res["knobs"],
                          "autotune": {"configurations": len(table), "best_ms_2_iterations": table[0]["ms_per_solve"],
                                       "worst_ms_2_iterations": table[-1]["ms_per_solve"]},
                          "frac_of_term_roofline": round(terms / (tb * 1e-3) / PEAK_TERMS_PER_S, 4)}
        bctx.close()
        log(f"[bench] batched (autotuned {tb_res['knobs']}) {tb:.3f} ms vs 64 plain {ts:.3f} ms (wall {tbw:.3f} vs "
            f"{tsw:.3f}); whole batched solve at {out['batched']['frac_of_term_roofline']:.3f} of the term roofline")

    # ---------------------------------------------------------------- adjoint: 8 x (forward + adjoint) per Adam step
    if not args.no_extra and args.only in (None, "adjoint"):
        bt = W.c5()
        T = int(bt.counts.sum())
        o = bt.offsets()
        ph = torch.rand(bt.b, bt.slm.ny, bt.slm.nx, device="cuda") * (2 * math.pi)
        G = torch.randn(T, 2, device="cuda")
        Vb = torch.empty(T, 2, device="cuda")
        gb = torch.empty_like(ph)

        def batched_fa():
            ctx.hot_forward_V(bt.slm, bt.counts, bt.xyz, ph, V=Vb)
            ctx.hot_adjoint(bt.slm, bt.counts, bt.xyz, ph, G, grad=gb)

        def plain_fa():
            for b in range(bt.b):
                ctx.hot_forward_V(bt.slm, [64], bt.xyz[o[b]:o[b + 1]], ph[b:b + 1], V=Vb[o[b]:o[b + 1]])
                ctx.hot_adjoint(bt.slm, [64], bt.xyz[o[b]:o[b + 1]], ph[b:b + 1], G[o[b]:o[b + 1]], grad=gb[b:b + 1])

        batched_fa()
        plain_fa()
        # both forms by wall clock with a final synchronisation (best of three runs of 10 steps) and
        # by HIP events on the stream (device time, including any gaps the host leaves); the plain
        # form is 16 calls that each upload a hologram's trap tables
        tb = min(time_wall(batched_fa, 10, sync) for _ in range(3))
        tp = min(time_wall(plain_fa, 10, sync) for _ in range(3))
        tbe = time_calls(batched_fa, 10, sync)
        tpe = time_calls(plain_fa, 10, sync)
        sync()
        h0 = time.perf_counter()
        for _ in range(10):
            plain_fa()
        host_ms = (time.perf_counter() - h0) / 10 * 1e3
        sync()
        # the workload's Adam step (lr 0.05): batched forward, loss, adjoint backward, Adam update
        phase0 = (torch.rand(bt.b, bt.slm.ny, bt.slm.nx, device="cuda") * (2 * math.pi)).contiguous()
        hot.optimize_phase(ctx, bt.slm, bt.counts, bt.xyz, phase0, steps=3, lr=0.05)
        sync()
        a0 = time.perf_counter()
        _, losses = hot.optimize_phase(ctx, bt.slm, bt.counts, bt.xyz, phase0, steps=50, lr=0.05)
        sync()
        adam_ms = (time.perf_counter() - a0) / 50 * 1e3
        upd = bt.slm.n * T
        out["adjoint"] = {"workload": f"{bt.name}: forward V + adjoint dL/dphi, 8 x 512^2 x 64 traps",
                          "ms": round(tb, 4), "updates_per_s": upd / (tb * 1e-3), "plain_ms": round(tp, 4),
                          "plain_updates_per_s": upd / (tp * 1e-3), "speedup_vs_plain": round(tp / tb, 3),
                          "device_ms": round(tbe, 4), "plain_device_ms": round(tpe, 4),
                          "speedup_vs_plain_device": round(tpe / tbe, 3),
                          "plain_host_enqueue_ms": round(host_ms, 4),
                          "adam_step_ms": round(adam_ms, 4),
                          "adam_loss_first_last_of_50": [round(float(losses[0]), 4), round(float(losses[-1]), 4)]}
        log(f"[bench] forward+adjoint batched {tb:.4f} ms vs plain {tp:.4f} ms wall, {tbe:.4f} vs {tpe:.4f} ms device "
            f"(plain host enqueue {host_ms:.4f} ms); Adam step {adam_ms:.3f} ms")

    # ---------------------------------------------------------------- stored exp(i Delta) variant (HBM-bound)
    if not args.no_extra and args.only in (None, "stored"):
        with hot.Context(0) as cs:
            cs.set_variant("stored")
            cs.hot_gsw(p.slm, p.xyz, p.theta0, K, phase=phase, V=V, stats=False)  # builds the 210 MB matrix

            def sstep():
                cs.hot_gsw(p.slm, p.xyz, p.theta0, K, phase=phase, V=V, stats=False)

            tsd = time_calls(sstep, 5, sync)
            pm = cs.hot_time_passes(p.slm, p.xyz, p.theta0, reps=20)
        bytes_pass = N * M * 8
        out["stored"] = {"workload": f"{p.name}, exp(i Delta) stored as complex64 [M][N] (210 MB)",
                         "ms_per_step": round(tsd, 4), "updates_per_s": N * M * K / (tsd * 1e-3),
                         "pass_ms": {"pixel": round(float(pm[2]), 5), "trap": round(float(pm[3]), 5)},
                         "pass_GBs": {"pixel": round(bytes_pass / (pm[2] * 1e-3) / 1e9, 1),
                                      "trap": round(bytes_pass / (pm[3] * 1e-3) / 1e9, 1)},
                         "hbm_peak_GBs": HBM_PEAK_GBS,
                         "note": "the 210 MB matrix fits the 256 MB MALL (last-level cache), so these pass rates "
                                 "are not HBM-bound; the 1024^2 x 256 line below (2.1 GB) is"}
        log(f"[bench] stored variant {tsd:.4f} ms/step")
        # the same variant with a matrix far larger than the MALL: HBM-bound passes
        q3 = W.c3()
        ph3 = torch.empty(q3.slm.ny, q3.slm.nx, device="cuda")
        V3 = torch.empty(q3.m, 2, device="cuda")
        with hot.Context(0) as cs:
            cs.set_variant("stored")
            cs.hot_gsw(q3.slm, q3.xyz, q3.theta0, q3.iters, phase=ph3, V=V3, stats=False)  # builds the matrix

            def sstep3():
                cs.hot_gsw(q3.slm, q3.xyz, q3.theta0, q3.iters, phase=ph3, V=V3, stats=False)

            tsd3 = time_calls(sstep3, 3, sync)
            pm3 = cs.hot_time_passes(q3.slm, q3.xyz, q3.theta0, reps=10)
        bytes3 = q3.slm.n * q3.m * 8
        out["stored"][q3.name] = {
            "workload": f"{q3.name}, exp(i Delta) stored as complex64 [M][N] ({bytes3 / 1e9:.2f} GB)",
            "ms_per_step": round(tsd3, 4), "updates_per_s": q3.slm.n * q3.m * q3.iters / (tsd3 * 1e-3),
            "pass_ms": {"pixel": round(float(pm3[2]), 5), "trap": round(float(pm3[3]), 5)},
            "pass_GBs": {"pixel": round(bytes3 / (pm3[2] * 1e-3) / 1e9, 1),
                         "trap": round(bytes3 / (pm3[3] * 1e-3) / 1e9, 1)}}
        del ph3, V3
        log(f"[bench] stored variant {q3.name}: {tsd3:.3f} ms/step; passes {bytes3 / (pm3[2] * 1e-3) / 1e9:.0f} "
            f"and {bytes3 / (pm3[3] * 1e-3) / 1e9:.0f} GB/s")

    # ---------------------------------------------------------------- separable reformulation (complex GEMMs)
    if not args.no_extra and args.only in (None, "separable"):
        res = {}
        with hot.Context(0) as cs:
            cs.set_variant("separable")
            for q in (W.c2(), W.c3()):
                ph = torch.empty(q.slm.ny, q.slm.nx, device="cuda")
                Vq = torch.empty(q.m, 2, device="cuda")

                def sstep():
                    cs.hot_gsw(q.slm, q.xyz, q.theta0, q.iters, phase=ph, V=Vq, stats=False)

                def sstep0():
                    cs.hot_gsw(q.slm, q.xyz, q.theta0, 0, phase=ph, V=Vq, stats=False)

                sstep()
                tsep = time_calls(sstep, 10, sync)
                sstep0()
                tsep0 = time_calls(sstep0, 10, sync)
                in_situ = (tsep - tsep0) / q.iters  # one fused launch per iteration
                pm = cs.hot_time_passes(q.slm, q.xyz, q.theta0, reps=20)
                flops = 16.0 * q.slm.n * q.m  # two complex contractions per iteration, 8 real flops per product
                ach = flops / (in_situ * 1e-3) / 1e12
                res[q.name] = {"ms_per_step": round(tsep, 4),
                               "updates_per_s": q.slm.n * q.m * q.iters / (tsep * 1e-3),
                               "speedup_vs_direct": None,
                               "ms_per_launch": {"iteration_in_situ": round(in_situ, 5),
                                                 "iteration_back_to_back": round(float(pm[0]), 5),
                                                 "collect_once_per_solve": round(float(pm[1]), 5),
                                                 "pixel_pass_alone": round(float(pm[2]), 5),
                                                 "trap_pass_alone": round(float(pm[3]), 5)},
                               "roofline": {"bound": "mfma",
                                            "kernel": "k_sep (update + both passes on FP32 MFMA + trap sums, fused)",
                                            "achieved": round(ach, 2), "peak": MFMA_F32_PEAK_TFLOPS,
                                            "unit": "TFLOP/s", "frac": round(ach / MFMA_F32_PEAK_TFLOPS, 4),
                                            "traffic": None}}
                log(f"[bench] separable {q.name}: {tsep:.4f} ms/step; iteration in situ {in_situ * 1e3:.2f} us, "
                    f"back to back {pm[0] * 1e3:.2f} us; pixel {pm[2]:.4f} trap {pm[3]:.4f}")
        if ms is not None and p.name in res:
            res[p.name]["speedup_vs_direct"] = round(ms / res[p.name]["ms_per_step"], 3)
        out["separable"] = {"note": "exact factorisation of Eq. 2, exp(i Delta) = X(column) Y(row): both passes as "
                                    "dense complex contractions on the FP32 matrix cores in one fused kernel per "
                                    "iteration; reported beside the direct-sum headline", **res}

    # ---------------------------------------------------------------- Fig. 7 analogue: quality at a 20 Hz frame budget
    if not args.no_extra and args.only in (None, "fig7"):
        fslm = W.Slm(768, 768)
        rows = []
        for n in range(2, 10):
            xyz = W.square_grid(n, 3e-6)
            th = W.random_phases(700 + n, n * n)
            fph = torch.empty(768, 768, device="cuda")
            fV = torch.empty(n * n, 2, device="cuda")
            ctx.hot_gsw(fslm, xyz, th, 20, phase=fph, V=fV, stats=False)
            t20 = time_calls(lambda: ctx.hot_gsw(fslm, xyz, th, 20, phase=fph, V=fV, stats=False), 5, sync)
            t_iter = t20 / 21.0  # 21 pixel + trap passes
            k_budget = int(min(50.0 / t_iter, 5000))
            st = ctx.hot_gsw(fslm, xyz, th, k_budget, phase=fph, V=fV, stats=True).stats
            rows.append({"traps": n * n, "grid": f"{n}x{n}", "ms_per_iteration": round(t_iter, 5),
                         "iterations_at_20Hz": k_budget,
                         "rs_e": round(float(st[0, 0]), 4), "rs_u": round(float(st[0, 1]), 4),
                         "gsw1_e": round(float(st[1, 0]), 4), "gsw1_u": round(float(st[1, 1]), 4),
                         "gsw20Hz_e": round(float(st[-1, 0]), 4), "gsw20Hz_u": round(float(st[-1, 1]), 4)})
        out["fig7"] = {"workload": "n x n planar grids (3 um pitch), 768^2 SLM; iterations that fit a 50 ms "
                                   "frame (capped at 5000)", "rows": rows}
        log("[bench] fig7 " + " ".join(f"{r['grid']}:K={r['iterations_at_20Hz']},u={r['gsw20Hz_u']}" for r in rows))

    # ---------------------------------------------------------------- interactive: rotating cube, 5 GSW iterations per frame
    if not args.no_extra and args.only in (None, "interactive"):
        from paper_0907_4027_amd.interactive import RealtimeLoop
        islm = W.Slm(1024, 768)
        loop = RealtimeLoop(ctx, islm, 8, iters=5)
        th0 = W.random_phases(600, 8)
        lat = []
        for f in range(96 + 4):
            frame, Vh, dt = loop.frame(W.rotating_cube(f, 96), th0)
            if f >= 4:
                lat.append(dt)
        lat = np.array(lat) * 1e3
        I = (Vh.numpy().astype(np.float64) ** 2).sum(1)
        out["interactive"] = {"workload": "rotating 5 um cube, 8 traps, 1024x768 SLM, 5 warm-started GSW iterations "
                                          "per frame, 8-bit frame copied to pinned host memory",
                              "frames": int(lat.size), "frame_ms_mean": round(float(lat.mean()), 4),
                              "frame_ms_p50": round(float(np.median(lat)), 4),
                              "frame_ms_p99": round(float(np.quantile(lat, 0.99)), 4),
                              "frames_per_s": round(float(1e3 / lat.mean()), 1),
                              "last_frame_efficiency": round(float(I.sum()), 4),
                              "last_frame_uniformity": round(float(1 - (I.max() - I.min()) / (I.max() + I.min())), 4)}
        log(f"[bench] interactive frame {lat.mean():.3f} ms mean, p99 {np.quantile(lat, 0.99):.3f} ms")

    # ---------------------------------------------------------------- measured pipe rates behind the roofline
    if args.only in (None, "peaks"):
        out["peaks"] = measure_peaks(ctx, log)

    # ---------------------------------------------------------------- CPU oracle on a bounded sample
    cpu = None
    if not args.no_cpu and args.only is None:
        import oracle
        Ks = 10
        t0 = time.perf_counter()
        oracle.solve("gsw", p.slm, p.xyz, p.theta0, Ks)
        dt = time.perf_counter() - t0
        # the same oracle on one thread, on a shorter sample (2 iterations, 6 passes)
        threads = oracle.get_threads()
        K1 = 2
        oracle.set_threads(1)
        t1 = time.perf_counter()
        oracle.solve("gsw", p.slm, p.xyz, p.theta0, K1)
        dt1 = time.perf_counter() - t1
        oracle.set_threads(threads)
        model = None
        try:
            with open("/proc/cpuinfo") as f:
                model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
        except OSError:
            pass
        cpu = {"value": N * M * Ks / dt, "unit": "pixel-trap updates/s", "cores": threads,
               "kind": "oracle", "sample": f"FP64 oracle GSW on the same 512^2 x 100 problem, {Ks} iterations "
                                           f"({2 * Ks + 2} passes), {dt:.2f} s",
               "one_thread": {"value": N * M * K1 / dt1, "sample": f"{K1} iterations ({2 * K1 + 2} passes), {dt1:.2f} s"},
               "host_cpu": model, "host_logical_cpus": os.cpu_count()}
        log(f"[bench] cpu oracle {dt:.2f} s for {Ks} iterations on {threads} threads; {dt1:.2f} s for {K1} "
            f"iterations on 1 thread ({model})")

    if ms is None:
        print(json.dumps({"section": args.only, **out, "roofline": roof, "tuning": tuning}))
        return
    value = N * M * K / (ms * 1e-3)
    line = {
        "metric": "pixel\u00b7trap updates/s, GSW 512\u00b2\u00d7100 3D traps; batched & adjoint vs plain",
        "value": value, "unit": "pixel\u00b7trap updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded trap arrays, workloads.c2)",
        "config": {"workload": "gsw-512sq-100traps", "nx": 512, "ny": 512, "traps": M, "iterations": K,
                   "algorithm": "GSW", "variant": "on-the-fly Delta", "parallelism": "single GPU",
                   "launch_shape": "library default"},
        "holograms_per_s": 1e3 / ms,
        "terms_per_s": 2 * N * M * (K + 1) / (ms * 1e-3),
        "end_to_end_ms": None if end_to_end_ms is None else round(end_to_end_ms, 4),
        "paper_context": {"updates_per_s": 1.34e9, "note": "the paper's GSW rate (0.44 ms per trap per iteration "
                          "at 768^2 on a GeForce GTX 260): other hardware and grid, not a target"},
        "roofline": roof, "cpu_baseline": cpu, "tuning": tuning, **out,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
