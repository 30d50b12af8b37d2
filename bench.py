#!/usr/bin/env python3
"""Benchmark: one full grid build per step on the 10M-triangle architectural scene.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

A step is one pass of the whole build (count + scan, expansion, radix sort,
ranges) over a device-resident scene, through the C ABI.  The line printed is
one JSON object with ms/build, Mpairs/s, the dominant kernel's HBM roofline
(its algorithmic bytes over its event-timed duration) and the CPU oracle's
rate on the same workload.  ``--batched`` adds the 512-grid batched build
against 512 one-at-a-time plain builds.

Other modes (for the counter calibration of profiles):
    python bench.py --mode copy      plain device copy of 1 GiB, 10 times
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E
PROFILES = os.path.join(ROOT, "profiles")


def kernel_bytes(name: str, T: int, NO: int, R: int) -> float:
    """Algorithmic bytes one launch of `name` must move (see the design doc for the model)."""
    return {
        "count_scan": 60.0 * T,            # 12 B indices + 36 B vertices in, 4 B start + 8 B box out
        "expand_hist": 12.0 * T + 8.0 * NO,  # start + box in, object-order pairs out
        "hist": 12.0 * T,                  # start + box of every object, keys regenerated
        "onesweep_expand": 12.0 * T + 8.0 * NO,  # regenerated keys in, pairs out
        "onesweep": 16.0 * NO,             # pairs in, pairs out
        "expand": 12.0 * T + 8.0 * NO,
        "ranges": 4.0 * NO + 8.0 * R,      # sorted cells in, (begin, end) per cell out
    }.get(name, 0.0)


def source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2403_10647_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it is current."""
    path = os.path.join(PROFILES, "traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(workload, {}).get(kernel)
    if not e or e.get("source_hash") != source_hash():
        return None
    return e.get("hbm_bytes_per_launch")


def cpu_baseline(scene, npairs: int) -> dict:
    import oracle
    assert oracle.probe_npairs(scene.verts, scene.tris, scene.lo, scene.hi, scene.res) == npairs
    t0 = time.perf_counter()
    c, o, r = oracle.build(scene.verts, scene.tris, scene.lo, scene.hi, scene.res, npairs=npairs)
    dt = time.perf_counter() - t0
    assert len(c) == npairs
    return {"value": round(npairs / dt / 1e6, 3), "unit": "Mpairs/s", "cores": 1, "kind": "oracle",
            "sample": f"the full workload, one serial build ({scene.ntris} triangles, {npairs} pairs) "
                      f"in {dt:.2f} s on {platform.processor() or platform.machine()}, {os.cpu_count()} host cores"}


def run_copy(steps: int):
    """A plain device copy of 1 GiB: the counter calibration and the practical HBM ceiling."""
    import torch
    n = 1 << 28  # 1 GiB of float32
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    print(json.dumps({"mode": "copy", "bytes_read_per_launch": 4 * n, "bytes_written_per_launch": 4 * n,
                      "launches": steps + 1, "ms_per_copy": round(ms, 4),
                      "GBps_read_plus_write": round(8 * n / (ms * 1e-3) / 1e9, 1)}), flush=True)


def run_batched(G, args) -> dict:
    """512-grid batched build against 512 one-at-a-time plain builds."""
    import numpy as np
    import torch
    from paper_2403_10647_amd import scenes
    t0 = time.time()
    batch = scenes.make_batch(args.seed, ngrids=args.ngrids)
    inputs = [G.GridInput.from_scene(s) for s in batch]
    gen_s = time.time() - t0
    ws_b = G.Workspace()
    caps = G.count_batched(inputs, ws_b)
    outs_b = G.alloc_results(inputs, caps)
    outs_p = G.alloc_results(inputs, caps)
    ws_p = G.Workspace()
    for _ in range(2):
        G.build_batched(inputs, outs_b, ws_b)
        for g, o in zip(inputs, outs_p):
            G.build(g, out=o, ws=ws_p)
    torch.cuda.synchronize()
    reps = max(1, args.batched_steps)
    t0 = time.perf_counter()
    for _ in range(reps):
        G.build_batched(inputs, outs_b, ws_b)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        for g, o in zip(inputs, outs_p):
            G.build(g, out=o, ws=ws_p)
    torch.cuda.synchronize()
    tp = (time.perf_counter() - t0) / reps
    same = all(torch.equal(a.cells[:a.npairs], b.cells[:b.npairs]) and torch.equal(a.objs[:a.npairs], b.objs[:b.npairs])
               and torch.equal(a.ranges, b.ranges) for a, b in zip(outs_b, outs_p))
    ntot = sum(caps)
    return {"ngrids": len(inputs), "triangles": int(sum(s.ntris for s in batch)), "npairs": int(ntot),
            "batched_builds_per_s": round(len(inputs) / tb, 1), "plain_builds_per_s": round(len(inputs) / tp, 1),
            "batched_ms": round(tb * 1e3, 3), "plain_ms": round(tp * 1e3, 3), "speedup": round(tp / tb, 3),
            "identical_outputs": bool(same), "generation_s": round(gen_s, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", default="arch", choices=["arch", "mixed", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched", action="store_true", help="also time the 512-grid batched build")
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--ngrids", type=int, default=512)
    ap.add_argument("--no-trace", action="store_true", help="time without per-kernel events")
    ap.add_argument("--mode", default="bench", choices=["bench", "copy"])
    ap.add_argument("--max-digit-bits", type=int, default=None, help="override the radix digit width")
    ap.add_argument("--fused", type=int, default=None, choices=[0, 1], help="first radix pass regenerates keys")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU; multi-GPU runs are not part of it (use --gpus 1)",
              file=sys.stderr, flush=True)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2403_10647_amd import _lib as G
    from paper_2403_10647_amd import scenes, stats

    if args.mode == "copy":
        run_copy(args.steps)
        return

    G.lib()
    torch.cuda.set_device(0)
    if args.max_digit_bits is not None:
        G.tune_set("max_digit_bits", args.max_digit_bits)
    if args.fused is not None:
        G.tune_set("fused_expand", args.fused)
    knobs = {"max_digit_bits": G.tune_get("max_digit_bits"), "fused_expand": G.tune_get("fused_expand")}
    t0 = time.time()
    scene = scenes.make_scene(args.workload, seed=args.seed)
    gin = G.GridInput.from_scene(scene)
    print(f"# scene {args.workload}: {scene.ntris} triangles, res {list(map(int, scene.res))}, "
          f"generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    ws = G.Workspace()
    npairs, _ = G.count(gin, ws)
    out = G.build(gin, cap_pairs=npairs, ws=ws)
    for _ in range(args.warmup):
        G.build(gin, ws=ws, out=out)
    torch.cuda.synchronize()

    trace = not args.no_trace
    if trace:
        G.trace_enable(True)
        G.trace_read()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        G.build(gin, ws=ws, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = G.trace_read() if trace else {}
    G.trace_enable(False)
    ms = wall * 1e3 / args.steps
    T, NO, R = scene.ntris, npairs, scene.ncells

    # the dominant kernel and its roofline
    dom = max(kern, key=lambda k: kern[k][1]) if kern else None
    roofline = None
    pipeline = None
    if dom:
        launches, tot_ms = kern[dom]
        avg_ms = tot_ms / launches
        bpl = kernel_bytes(dom, T, NO, R)
        achieved = bpl / (avg_ms * 1e-3) / 1e9
        traffic = load_traffic(dom, args.workload)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                    "avg_launch_ms": round(avg_ms, 5), "bytes_per_launch": int(bpl)}
        b_alg = sum(kernel_bytes(k, T, NO, R) * v[0] for k, v in kern.items()) / args.steps
        kern_ms = sum(v[1] for v in kern.values()) / args.steps
        pipeline = {"bytes_alg_per_build": int(b_alg), "frac_of_peak_at_ms_per_build": round(b_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "kernel_ms_per_build": round(kern_ms, 4),
                    "kernels": {k: {"launches_per_build": v[0] / args.steps, "avg_ms": round(v[1] / v[0], 5)}
                                for k, v in sorted(kern.items(), key=lambda kv: -kv[1][1])}}

    c_np = out.ranges.cpu().numpy().view(np.uint32)
    row = stats.table1_from_ranges(scene.res, T, c_np, np.array([0]))
    result = {
        "metric": "ms/build + Mpairs/s at 10M tris (% HBM roofline); batched builds/s vs plain",
        "value": round(NO / (ms * 1e-3) / 1e6, 2),
        "unit": "Mpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "ms_per_build": round(ms, 4),
        "builds_per_s": round(1e3 / ms, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: " + {
            "arch": "10M-triangle architectural-style soup (10k wall rectangles + 2000 Gaussian clusters) in a "
                    "100x10x100 box, lambda=2, cap 1024",
            "mixed": "1M triangles, 95% small / 5% large, lambda=4, cap 512",
            "small": "4096 small triangles, 32^3 grid"}[args.workload],
                   "knobs": knobs, "triangles": T, "npairs": NO, "res": [int(x) for x in scene.res], "cells": R, "seed": args.seed,
                   "table1": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in row.items()
                              if k not in ("max_cells_per_item",)}},
        "event_ms_per_build": round(ev0.elapsed_time(ev1) / args.steps, 4),
        "roofline": roofline,
        "pipeline": pipeline,
        "cpu_baseline": None,
    }
    if args.batched:
        result["batched"] = run_batched(G, args)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(scene, NO)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
