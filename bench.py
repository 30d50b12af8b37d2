#!/usr/bin/env python3
"""Benchmark: one full grid build per step on the 10M-triangle architectural scene.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

A step is one pass of the whole build (count + scan, expansion, radix sort,
ranges) over a device-resident scene, through the C ABI.  The line printed is
one JSON object with ms/build, Mpairs/s, the dominant kernel's HBM roofline
(its algorithmic bytes over its event-timed duration) and the CPU oracle's
rate on the same workload, with the GPU grid compared to the oracle's grid.
Unless switched off it also times the 512-grid batched build (eager and as a
replayed graph) against 512 one-at-a-time plain builds, and serves Poisson
arrivals of requests shaped like those grids, plus the 10M-triangle scene once a
second, through the continuous-batching server (p50/p99 latency, builds/s).

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
    """Algorithmic bytes one launch of `name` must move: each input read once and
    each output written once, for T triangles, NO pairs and R cells (look-back
    words, histograms and re-reads are not counted)."""
    return {
        "count_scan": 60.0 * T,            # 12 B indices + 36 B vertices in, 4 B start + 8 B box out
        "expand_hist": 12.0 * T + 8.0 * NO,  # start + box in, object-order pairs out
        "hist": 12.0 * T,                  # start + box of every object, keys regenerated
        "onesweep_expand": 12.0 * T + 8.0 * NO,  # regenerated keys in, pairs out
        "onesweep": 16.0 * NO,             # pairs in, pairs out
        "expand": 12.0 * T + 8.0 * NO,
        "ranges": 4.0 * NO + 8.0 * R,      # sorted cells in, (begin, end) per cell out
    }.get(name, 0.0)


def survey_bytes(T: int, NO: int, R: int, passes: int) -> int:
    """The unfused per-build byte model, at the radix passes the build runs:
    80 T + (16 + 16 P) NO + 8 R (inputs, count/start and box round trips, the
    expansion's pairs, one histogram read, P passes that read and write key and
    value, the range pass's read of the sorted cells, and the range table)."""
    return 80 * T + (16 + 16 * passes) * NO + 8 * R


def source_hash() -> str:
    """Hash of the kernel sources' code (comments and whitespace left out), which
    ties the committed traffic counters to the kernels they were taken on."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2403_10647_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(f.encode() + " ".join(text.split()).encode())
    return h.hexdigest()[:16]


def knobs_key(knobs: dict) -> str:
    return ",".join(f"{k}={int(knobs[k])}" for k in ("max_digit_bits", "sort_shape", "fused_expand"))


def load_traffic(kernel: str, workload: str, knobs: dict):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it was taken at
    these knobs and is current."""
    path = os.path.join(PROFILES, "traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(workload, {}).get(knobs_key(knobs), {}).get(kernel)
    if not e or e.get("source_hash") != source_hash():
        return None
    return e.get("hbm_bytes_per_launch")


def cpu_baseline(scene, gpu_out) -> dict:
    """The oracle timed on one host core over the whole workload; its grid is then compared
    with the GPU's, element by element."""
    import numpy as np
    import oracle
    no = oracle.probe_npairs(scene.verts, scene.tris, scene.lo, scene.hi, scene.res)  # sizes the oracle's output
    times = []
    for _ in range(3):   # the median of three whole serial builds
        t0 = time.perf_counter()
        c, o, r = oracle.build(scene.verts, scene.tris, scene.lo, scene.hi, scene.res, npairs=no)
        times.append(time.perf_counter() - t0)
    dt = sorted(times)[1]
    npairs = int(no)
    gc, go, gr = gpu_out.numpy()
    same = bool(gpu_out.npairs == npairs and np.array_equal(c, gc) and np.array_equal(o, go) and np.array_equal(r, gr))
    return {"value": round(npairs / dt / 1e6, 3), "unit": "Mpairs/s", "cores": 1, "kind": "oracle",
            "sample": f"the full workload, median of three serial builds ({scene.ntris} triangles, {npairs} pairs): "
                      f"{dt:.2f} s (runs {', '.join(f'{x:.2f}' for x in times)} s) on "
                      f"{platform.processor() or platform.machine()}, {os.cpu_count()} host cores",
            "gpu_grid_identical": same}


def run_copy(steps: int):
    """Counter calibration and the practical HBM ceiling: a plain device copy of 1 GiB, then the same
    1 GiB moved as 128-byte rows in a random order, read by a gather (index_select) and written by a
    scatter (index_copy_), whose HBM bytes are as exact as the copy's: every row is read once and
    written once, whole, plus the 8-byte row indices."""
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
    out = {"mode": "copy", "bytes_read_per_launch": 4 * n, "bytes_written_per_launch": 4 * n,
           "launches": steps + 1, "ms_per_copy": round(ms, 4),
           "GBps_read_plus_write": round(8 * n / (ms * 1e-3) / 1e9, 1)}
    rows = n // 32  # 128-byte rows
    a2, b2 = a.view(rows, 32), b.view(rows, 32)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    perm = torch.randperm(rows, device="cuda", generator=gen)
    for name, fn in (("gather_rows", lambda: torch.index_select(a2, 0, perm, out=b2)),
                     ("scatter_rows", lambda: b2.index_copy_(0, perm, a2))):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = {"bytes_read_per_launch": 4 * n + 8 * rows, "bytes_written_per_launch": 4 * n,
                     "ms": round(e0.elapsed_time(e1) / steps, 4)}
    print(json.dumps(out), flush=True)


def run_configs(G, args, steps: int = 20) -> dict:
    """The other single-grid configurations: the 4096-triangle scene (launch
    bound: microseconds per build) and the 1M mixed scene (ms per build,
    Mpairs/s, the dominant kernel's roofline and the unfused byte model's fraction)."""
    import torch
    from paper_2403_10647_amd import scenes
    res = {}
    for name in ("small", "mixed"):
        s = scenes.make_scene(name, seed=args.seed)
        g = G.GridInput.from_scene(s)
        ws = G.Workspace()
        n, _ = G.count(g, ws)
        out = G.build(g, cap_pairs=n, ws=ws)
        b = G.PlainBuild(g, out, ws)
        for _ in range(3):
            b()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            b()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        G.trace_enable(True)
        G.trace_read()
        for _ in range(steps):
            b()
        k = G.trace_read()
        G.trace_enable(False)
        T, R = s.ntris, s.ncells
        dom = max(k, key=lambda x: k[x][1])
        avg = k[dom][1] / k[dom][0]
        bpl = kernel_bytes(dom, T, n, R)
        passes = G.sort_plan(max(0, (R - 1).bit_length()))[0]
        bs = survey_bytes(T, n, R, passes)
        res[name] = {"triangles": T, "npairs": n, "cells": R, "ms_per_build": round(ms, 4),
                     "us_per_build": round(ms * 1e3, 1), "Mpairs_per_s": round(n / (ms * 1e-3) / 1e6, 1),
                     "radix_passes": passes, "bytes_survey_model": int(bs),
                     "frac_survey_model": round(bs / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "roofline": {"kernel": dom, "avg_launch_ms": round(avg, 5), "bytes_per_launch": int(bpl),
                                  "achieved": round(bpl / (avg * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                                  "frac": round(bpl / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
                     "kernels_ms": {x: round(v[1] / steps, 4) for x, v in sorted(k.items(), key=lambda kv: -kv[1][1])}}
        del b, out, ws
    torch.cuda.empty_cache()
    return res


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
    # both sides marshal their C arguments once: one C call per batch, one per plain build
    batch_build = G.BatchedBuild(inputs, outs_b, ws_b)
    ws_p.get(max(G.workspace_size(g.ntris, c, g.res) for g, c in zip(inputs, caps)))
    plain_builds = [G.PlainBuild(g, o, ws_p) for g, o in zip(inputs, outs_p)]
    for _ in range(2):
        batch_build()
        for b in plain_builds:
            b()
    torch.cuda.synchronize()
    reps = max(1, args.batched_steps)
    t0 = time.perf_counter()
    for _ in range(reps):
        batch_build()
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        for b in plain_builds:
            b()
    torch.cuda.synchronize()
    tp = (time.perf_counter() - t0) / reps
    # one more batched build with per-kernel events, outside the timed region
    G.trace_enable(True)
    G.trace_read()
    G.build_batched(inputs, outs_b, ws_b)
    kern = G.trace_read()
    G.trace_enable(False)
    batched_kernels = {k: {"launches": v[0], "ms": round(v[1], 4)} for k, v in sorted(kern.items(), key=lambda kv: -kv[1][1])}
    # the same batch as one captured graph of the asynchronous build, replayed
    outs_g = G.alloc_results(inputs, caps)
    ws_g = G.Workspace()
    stage = torch.empty(int(G.lib().grid_batch_staging_size(len(inputs))), dtype=torch.uint8, pin_memory=True)
    sg = torch.cuda.Stream()
    G.build_batched_async(inputs, outs_g, caps, ws_g, stage, stream=sg)
    sg.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=sg):
        G.build_batched_async(inputs, outs_g, caps, ws_g, stage, stream=sg)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        graph.replay()
    torch.cuda.synchronize()
    tg = (time.perf_counter() - t0) / reps
    g_status = G.workspace_status(ws_g)[0]

    def same_as_plain(outs):
        return all(torch.equal(a.cells[:a.npairs], b.cells[:b.npairs]) and torch.equal(a.objs[:a.npairs], b.objs[:b.npairs])
                   and torch.equal(a.ranges, b.ranges) for a, b in zip(outs, outs_p))
    same = same_as_plain(outs_b)
    same_g = g_status == G.GRID_OK and same_as_plain(outs_g)
    ntot = sum(caps)
    cells_tot = sum(g.ncells for g in inputs)
    plan = G.sort_plan(max(1, (cells_tot - 1).bit_length()))
    b_survey = sum(survey_bytes(s.ntris, c, s.ncells, plan[0]) for s, c in zip(batch, caps))
    sweeps = [(k, v) for k, v in kern.items() if k.startswith("onesweep")]
    sw_launch, sw_ms = sum(v[0] for _, v in sweeps), sum(v[1] for _, v in sweeps)
    batch_roof = None
    if sw_launch:
        avg = sw_ms / sw_launch
        batch_roof = {"kernel": "onesweep (all passes)", "avg_launch_ms": round(avg, 5),
                      "bytes_per_launch": 16 * int(ntot), "achieved": round(16 * ntot / (avg * 1e-3) / 1e9, 1),
                      "peak": HBM_PEAK_GBS, "frac": round(16 * ntot / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    res = {"ngrids": len(inputs), "triangles": int(sum(s.ntris for s in batch)), "npairs": int(ntot),
           "cells": int(cells_tot), "bytes_survey_model": int(b_survey),
           "frac_survey_model": round(b_survey / tb / 1e9 / HBM_PEAK_GBS, 4), "roofline": batch_roof,
           "batched_builds_per_s": round(len(inputs) / tb, 1), "plain_builds_per_s": round(len(inputs) / tp, 1),
           "graph_builds_per_s": round(len(inputs) / tg, 1),
           "batched_ms": round(tb * 1e3, 3), "graph_ms": round(tg * 1e3, 3), "plain_ms": round(tp * 1e3, 3),
           "speedup": round(tp / tb, 3), "graph_speedup": round(tp / tg, 3),
           "identical_outputs": bool(same), "graph_identical_outputs": bool(same_g), "generation_s": round(gen_s, 1),
           "sort_plan": G.sort_plan(max(1, (sum(g.ncells for g in inputs) - 1).bit_length())),
           "kernels": batched_kernels}
    del outs_b, outs_g, ws_g, ws_b
    torch.cuda.empty_cache()
    return res, inputs, outs_p


def run_ablation(G, args, gin, out, ws, reps: int = 5) -> dict:
    """Pair generation one thread per pair (the per-pair expansion of the
    paper's method) against one thread per object (the MakePairs of sorted-grid
    builders), with the same sort and ranges after it, on the headline scene and
    on the 1M mixed scene whose 5% large triangles hold most of its pairs.
    Outputs are compared bit for bit with the default build's."""
    import torch
    from paper_2403_10647_amd import scenes
    mixed = G.GridInput.from_scene(scenes.make_scene("mixed", seed=args.seed))
    n_mixed, _ = G.count(mixed, ws)
    cases = [(args.workload, gin, out), ("mixed", mixed, G.build(mixed, cap_pairs=n_mixed, ws=ws))]
    res = {}
    for name, g, ref in cases:
        n = ref.npairs
        row = {"triangles": g.ntris, "npairs": n}
        for knob, label, gen in ((0, "per_pair", "expand_hist"), (1, "per_object", "makepairs_hist")):
            G.tune_set("per_object_pairs", knob)
            try:
                o = G.build(g, cap_pairs=n, ws=ws)
                run = G.PlainBuild(g, o, ws)
                run()
                torch.cuda.synchronize()
                G.trace_enable(True)
                G.trace_read()
                t0 = time.perf_counter()
                for _ in range(reps):
                    run()
                torch.cuda.synchronize()
                wall = (time.perf_counter() - t0) * 1e3 / reps
                k = G.trace_read()
            finally:
                G.trace_enable(False)
                G.tune_set("per_object_pairs", 0)
            same = (torch.equal(o.cells[:n], ref.cells[:n]) and torch.equal(o.objs[:n], ref.objs[:n])
                    and torch.equal(o.ranges, ref.ranges))
            row[label] = {"ms_per_build": round(wall, 4),
                          "pair_generation_ms": round(k[gen][1] / k[gen][0], 4) if gen in k else None,
                          "identical_to_default": bool(same)}
            del o, run
        a, b = row["per_pair"]["pair_generation_ms"], row["per_object"]["pair_generation_ms"]
        row["per_object_over_per_pair"] = round(b / a, 2) if a and b else None
        res[name] = row
    return res


def run_culled(G, args, gin, out, ws, reps: int = 5) -> dict:
    """The build with false intersections removed (grid_build_culled) against the
    plain build on the headline scene, the 1M mixed scene and a 1M-triangle
    Hairball-like scene of long thin diagonal slivers: box and kept pair counts
    and ms per build, both timed as repeated calls on resident buffers."""
    import torch
    from paper_2403_10647_amd import scenes
    cases = [(args.workload, gin, out)]
    for name in ("mixed", "hairball"):
        g = G.GridInput.from_scene(scenes.make_scene(name, seed=args.seed))
        n, _ = G.count(g, ws)
        cases.append((name, g, G.build(g, cap_pairs=n, ws=ws)))
    res = {}
    for name, g, ref in cases:
        nbox = ref.npairs
        plain = G.PlainBuild(g, ref, ws)
        o, _ = G.build_culled(g, box_cap=nbox, ws=ws)
        culled = G.CulledBuild(g, o, nbox, ws)
        row = {"triangles": g.ntris, "box_npairs": nbox}
        for label, fn in (("plain", plain), ("culled", culled)):
            fn()
            torch.cuda.synchronize()
            G.trace_enable(True)
            G.trace_read()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            row[f"{label}_ms_per_build"] = round((time.perf_counter() - t0) * 1e3 / reps, 4)
            k = G.trace_read()
            G.trace_enable(False)
            row[f"{label}_kernels"] = {kk: round(v[1] / reps, 4) for kk, v in k.items()}
        row["kept_npairs"] = o.npairs
        row["kept_fraction"] = round(o.npairs / max(nbox, 1), 4)
        row["ms_saved"] = round(row["plain_ms_per_build"] - row["culled_ms_per_build"], 4)
        res[name] = row
        del plain, culled, o
    return res


def run_paths(G, args, gin, out, ws, reps: int = 5) -> dict:
    """The sorted path against the compact path (atomic counting scatter plus
    in-cell sorts) of grid_build on homogeneous and non-homogeneous scenes, and
    the path the statistics pass picks (build_path = 2) with its time; every
    path's grid is compared with the sorted path's on the device."""
    import torch
    from paper_2403_10647_amd import scenes
    cases = [("small", None), ("uniform", 16_384), ("uniform", 65_536), ("uniform", 262_144), ("uniform", 1_000_000),
             ("uniform", 4_000_000), ("mixed", None), ("hairball", None)]
    res = {}
    todo = [(args.workload, gin, out)]
    for name, n in cases:
        s = scenes.make_scene(name, seed=args.seed, ntris=n)
        g = G.GridInput.from_scene(s)
        no, _ = G.count(g, ws)
        todo.append((f"{name}_{s.ntris}", g, G.build(g, cap_pairs=no, ws=ws)))
    for label, g, ref in todo:
        n = ref.npairs
        row = {"triangles": g.ntris, "npairs": n, "cells": g.ncells, "pairs_per_cell": round(n / g.ncells, 3)}
        o = G.build(g, cap_pairs=n, ws=ws)
        for path, key in ((0, "sorted"), (1, "compact"), (2, "auto")):
            G.tune_set("build_path", path)
            try:
                run = G.PlainBuild(g, o, ws)
                run()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    run()
                torch.cuda.synchronize()
                row[f"{key}_ms"] = round((time.perf_counter() - t0) * 1e3 / reps, 4)
                if path == 2:
                    row["auto_path"] = ("sorted", "compact")[G.tune_get("last_path")]
                if path == 1:  # where the compact path's time goes (a separate traced build)
                    G.trace_enable(True)
                    G.trace_read()
                    run()
                    row["compact_kernels_ms"] = {kk: round(v[1], 4) for kk, v in G.trace_read().items()}
                    G.trace_enable(False)
                row[f"{key}_identical"] = bool(torch.equal(o.cells[:n], ref.cells[:n]) and torch.equal(o.objs[:n], ref.objs[:n])
                                               and torch.equal(o.ranges, ref.ranges))
            finally:
                G.tune_set("build_path", 0)
        row["compact_over_sorted"] = round(row["compact_ms"] / row["sorted_ms"], 3)
        res[label] = row
        del o
    return res


def time_raycast(G, g, grid, rays, reps: int = 3):
    """ms for one grid_raycast of the rays over the grid (event-timed, after a warm-up) and the hit count."""
    import torch
    ht, ho = G.raycast(g, grid, rays)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        G.raycast(g, grid, rays)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, int((ho != -1).sum().item())


def run_raycast(G, args, scene, gin, out, ws, nrays: int = 1 << 20) -> dict:
    """Closest-hit ray casting over the headline grid (the query the grid is
    built for): 1M seeded rays (70% starting inside the box in uniform
    directions, 30% aimed in from outside), over the sorted grid and over the
    culled grid of the same scene, with the outputs of the two compared."""
    import torch
    from paper_2403_10647_amd import scenes
    rays = torch.from_numpy(scenes.make_rays(scene, nrays, seed=args.seed)).cuda()
    ms, hits = time_raycast(G, gin, out, rays)
    ht, ho = G.raycast(gin, out, rays)
    nbox = out.npairs
    culled, _ = G.build_culled(gin, box_cap=nbox, ws=ws)
    ms_c, _ = time_raycast(G, gin, culled, rays)
    ct, co = G.raycast(gin, culled, rays)
    same = bool(torch.equal(ht.view(torch.int32), ct.view(torch.int32)) and torch.equal(ho, co))
    del culled
    return {"rays": nrays, "hits": hits, "ms": round(ms, 4), "Mrays_per_s": round(nrays / (ms * 1e-3) / 1e6, 1),
            "culled_grid_ms": round(ms_c, 4), "culled_grid_Mrays_per_s": round(nrays / (ms_c * 1e-3) / 1e6, 1),
            "culled_grid_identical_hits": same}


def run_resolution(G, args, reps: int = 5) -> dict:
    """The cell-size rule revisited (the paper leaves it open): the sorted build
    of the 10M arch scene and the 1M mixed scene at lambda = 1, 2, 4, 8 cells
    per triangle (the resolution rule's parameter), with the pair count, the
    cells, the build time and the time to cast 256K seeded rays over the grid
    (scaled to 1M rays) at each: finer cells cost build time and save query time."""
    import torch
    from paper_2403_10647_amd import scenes
    res = {}
    for name, cap in (("arch", 1024), ("mixed", 512)):
        s = scenes.make_scene(name, seed=args.seed)
        base = G.GridInput.from_scene(s)
        rays = torch.from_numpy(scenes.make_rays(s, 1 << 18, seed=args.seed)).cuda()
        rows = {}
        for lam in (1.0, 2.0, 4.0, 8.0):
            r = scenes.resolution_rule(s.lo, s.hi, s.ntris, lam, cap)
            g = G.GridInput(base.verts, base.tris, list(map(float, s.lo)), list(map(float, s.hi)), list(map(int, r)))
            ws = G.Workspace()
            n, _ = G.count(g, ws)
            out = G.build(g, cap_pairs=n, ws=ws)
            b = G.PlainBuild(g, out, ws)
            b()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                b()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / reps
            rms, hits = time_raycast(G, g, out, rays)
            rows[f"lambda_{lam:g}"] = {"res": [int(x) for x in r], "cells": g.ncells, "npairs": n,
                                       "pairs_per_triangle": round(n / s.ntris, 3), "ms_per_build": round(ms, 4),
                                       "raycast_ms_per_1M_rays": round(rms * (1 << 20) / rays.shape[1], 4),
                                       "hits": hits}
            del b, out, ws, g
        res[name] = rows
        torch.cuda.empty_cache()
    return res


def run_served(G, args, pool, pool_refs, big, big_ref) -> dict:
    """Poisson arrivals of requests drawn from the batch's grids plus the 10M-triangle scene once a
    second, through the continuous-batching server; every output is compared on the device with the
    same scene's stand-alone build.  Then the same kind of requests all at once (burst), under the
    full budget and under a tight one, against one-at-a-time plain builds."""
    import torch
    from paper_2403_10647_amd import serve
    refs = list(pool_refs) + [big_ref]
    big_key = len(pool)
    ws = serve.batch_workspace_bytes([big], [big_ref.npairs])
    budget = args.serve_budget_gb << 30
    srv = serve.Server(budget, ws, nslots=args.serve_slots, max_pairs=args.serve_max_pairs, references=refs)
    warm = serve.make_requests(pool, rate=2000.0, duration=0.2, seed=args.seed + 100, big=big, big_key=big_key)
    srv.run(warm)
    reqs = serve.make_requests(pool, rate=args.serve_rate, duration=args.serve_seconds, seed=args.seed, big=big,
                               big_every=1.0, big_key=big_key)
    print(f"# serving {len(reqs)} requests over {args.serve_seconds} s", file=sys.stderr, flush=True)
    st = srv.run(reqs).as_dict()
    # requests one at a time: one every millisecond, each done long before the next arrives
    lone = srv.run(serve.spaced_requests(pool, gap=1e-3, count=1000, seed=args.seed + 2)).as_dict()
    burst = serve.make_requests(pool, rate=2000.0, duration=1.0, seed=args.seed + 1, big=big, big_key=big_key,
                                burst=True)
    srv.run(burst)                      # untimed: sizes the allocator's blocks for batches this large
    sb = srv.run(burst).as_dict()
    del srv
    torch.cuda.empty_cache()
    big_out = serve.output_bytes(big_ref.npairs, big.ncells)
    tight = 2 * ws + big_out + (256 << 20)
    srv_t = serve.Server(tight, ws, nslots=2, max_pairs=args.serve_max_pairs, references=refs)
    srv_t.run(burst)
    stt = srv_t.run(burst).as_dict()
    del srv_t
    torch.cuda.empty_cache()
    plain = serve.plain_builds_per_s(burst)
    ok = st["mismatches"] == 0 and sb["mismatches"] == 0 and stt["mismatches"] == 0 and lone["mismatches"] == 0
    return {"open_loop": {"rate_per_s": args.serve_rate, "big_every_s": 1.0, **st},
            "lone": {"gap_ms": 1.0, **{k: lone[k] for k in ("requests", "completed", "p50_ms", "p99_ms",
                                                                    "max_ms", "mean_batch", "mismatches")}},
            "burst": sb, "burst_tight_budget": stt,
            "burst_plain_builds_per_s": round(plain["builds_per_s"], 1),
            "burst_speedup_vs_plain": round(sb["builds_per_s"] / plain["builds_per_s"], 3),
            "slot_workspace_bytes": ws, "all_outputs_identical_to_alone": bool(ok)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", default="arch", choices=["arch", "mixed", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-grid batched build and serving")
    ap.add_argument("--no-serve", action="store_true", help="skip serving")
    ap.add_argument("--no-culled", action="store_true", help="skip the culled-build comparison")
    ap.add_argument("--no-configs", action="store_true", help="skip the small and mixed single-grid configurations")
    ap.add_argument("--no-paths", action="store_true", help="skip the sorted/compact path comparison")
    ap.add_argument("--no-resolution", action="store_true", help="skip the cell-size (lambda) sweep")
    ap.add_argument("--no-raycast", action="store_true", help="skip ray casting over the headline grid")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the per-object pair generation comparison")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-budget-gb", type=int, default=64)
    ap.add_argument("--serve-slots", type=int, default=3)
    ap.add_argument("--serve-max-pairs", type=int, default=1 << 25)
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--ngrids", type=int, default=512)
    ap.add_argument("--no-trace", action="store_true", help="time without per-kernel events")
    ap.add_argument("--mode", default="bench", choices=["bench", "copy"])
    ap.add_argument("--max-digit-bits", type=int, default=None, help="override the radix digit width")
    ap.add_argument("--fused", type=int, default=None, choices=[0, 1], help="first radix pass regenerates keys")
    ap.add_argument("--sort-shape", type=int, default=None, help="radix pass workgroup shape (grid_tune_set sort_shape)")
    ap.add_argument("--no-tune", action="store_true",
                    help="time the headline build with the default knobs instead of the tuner's choice")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; multi-GPU runs are not supported (use --gpus 1)",
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
    if args.sort_shape is not None:
        G.tune_set("sort_shape", args.sort_shape)
    t0 = time.time()
    scene = scenes.make_scene(args.workload, seed=args.seed)
    gin = G.GridInput.from_scene(scene)
    print(f"# scene {args.workload}: {scene.ntris} triangles, res {list(map(int, scene.res))}, "
          f"generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    # the headline build runs the tuner's choice for this scene (every candidate's grid is checked
    # against the default's), confirmed against the defaults in alternating rounds
    tuning = None
    explicit = args.max_digit_bits is not None or args.fused is not None or args.sort_shape is not None
    if not args.no_tune and not explicit:
        from paper_2403_10647_amd import tune
        print("# tuning", file=sys.stderr, flush=True)
        best, table = tune.tune_plain(gin, reps=5, G=G)
        chosen, med = tune.confirm_plain(gin, best, G=G)
        tune.set_knobs(G, chosen)
        tuning = {"candidates": len(table), "all_identical_grids": all(r["identical"] for r in table),
                  "search_best": best, "confirm_median_ms": med, "chosen": chosen,
                  "top3": [{"knobs": r["knobs"], "ms": r["ms"]} for r in table[:3]]}
        torch.cuda.empty_cache()
    knobs = {k: G.tune_get(k) for k in ("max_digit_bits", "fused_expand", "sort_shape")}
    ws = G.Workspace()
    npairs, _ = G.count(gin, ws)
    out = G.build(gin, cap_pairs=npairs, ws=ws)
    build = G.PlainBuild(gin, out, ws)   # grid_build with its arguments marshalled once
    for _ in range(args.warmup):
        build()
    torch.cuda.synchronize()

    # per-kernel breakdown: K traced builds, every kernel bracketed by events
    T, NO, R = scene.ntris, npairs, scene.ncells
    G.trace_enable(True)
    G.trace_read()
    for _ in range(args.steps):
        build()
    torch.cuda.synchronize()
    kern_all = G.trace_read()
    G.trace_enable(False)
    dom = max(kern_all, key=lambda k: kern_all[k][1]) if kern_all else None

    # the timed region: K builds; events bracket only the dominant kernel's
    # launches (on the stream they are launched on), for its roofline.  When
    # that kernel is the radix pass, one pair of events spans a build's passes
    # (which run back to back), so that the timed builds carry two event
    # records each instead of two per pass
    trace = not args.no_trace and dom is not None
    span = dom == "onesweep" and all(k == "onesweep" or not k.startswith("onesweep") for k in kern_all)
    if trace:
        G.trace_only("radix_passes" if span else dom)
        G.trace_enable(True)
        G.trace_read()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        build()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = G.trace_read() if trace else {}
    G.trace_enable(False)
    G.trace_only(None)
    ms = wall * 1e3 / args.steps

    roofline = None
    pipeline = None
    if dom:
        if span and "radix_passes" in kern:
            # the span's total over the passes it covers
            launches, tot_ms = kern_all[dom][0], kern["radix_passes"][1]
        else:
            launches, tot_ms = kern[dom] if dom in kern else kern_all[dom]
        avg_ms = tot_ms / launches
        bpl = kernel_bytes(dom, T, NO, R)
        achieved = bpl / (avg_ms * 1e-3) / 1e9
        traffic = load_traffic(dom, args.workload, knobs)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                    "avg_launch_ms": round(avg_ms, 5), "bytes_per_launch": int(bpl),
                    "events": ("timed region, one span over each build's passes" if span and "radix_passes" in kern
                               else "timed region" if dom in kern else "separate traced run")}
        b_alg = sum(kernel_bytes(k, T, NO, R) * v[0] for k, v in kern_all.items()) / args.steps
        kern_ms = sum(v[1] for v in kern_all.values()) / args.steps
        passes = G.sort_plan(max(0, (R - 1).bit_length()))[0]
        b_survey = survey_bytes(T, NO, R, passes)
        pipeline = {"bytes_alg_per_build": int(b_alg), "frac_of_peak_at_ms_per_build": round(b_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "radix_passes": passes, "bytes_survey_model": int(b_survey),
                    "frac_survey_model": round(b_survey / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "kernel_ms_per_build": round(kern_ms, 4),
                    "kernels": {k: {"launches_per_build": v[0] / args.steps, "avg_ms": round(v[1] / v[0], 5)}
                                for k, v in sorted(kern_all.items(), key=lambda kv: -kv[1][1])}}

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
                   "knobs": knobs, "tuning": tuning, "triangles": T, "npairs": NO, "res": [int(x) for x in scene.res], "cells": R, "seed": args.seed,
                   "table1": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in row.items()
                              if k not in ("max_cells_per_item",)}},
        "event_ms_per_build": round(ev0.elapsed_time(ev1) / args.steps, 4),
        "roofline": roofline,
        "pipeline": pipeline,
        "cpu_baseline": None,
    }
    if tuning is not None:
        # the other sections measure the default knobs
        from paper_2403_10647_amd import tune
        tune.set_knobs(G, tune.DEFAULTS)
    if not args.no_configs:
        print("# configurations", file=sys.stderr, flush=True)
        result["configs"] = run_configs(G, args)
    if not args.no_batched:
        print("# batched", file=sys.stderr, flush=True)
        result["batched"], pool, pool_refs = run_batched(G, args)
        if not args.no_serve:
            print("# serving", file=sys.stderr, flush=True)
            result["served"] = run_served(G, args, pool, pool_refs, gin, out)
        del pool, pool_refs
    if not args.no_paths:
        print("# sorted and compact paths", file=sys.stderr, flush=True)
        result["paths"] = run_paths(G, args, gin, out, ws)
    if not args.no_raycast:
        print("# ray casting", file=sys.stderr, flush=True)
        result["raycast"] = run_raycast(G, args, scene, gin, out, ws)
    if not args.no_resolution:
        print("# resolution sweep", file=sys.stderr, flush=True)
        result["resolution"] = run_resolution(G, args)
    if not args.no_culled:
        print("# culled builds", file=sys.stderr, flush=True)
        result["culled"] = run_culled(G, args, gin, out, ws)
    if not args.no_ablation:
        print("# per-object pair generation", file=sys.stderr, flush=True)
        result["ablation"] = run_ablation(G, args, gin, out, ws)
    if not args.no_cpu_baseline:
        print("# cpu baseline", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(scene, out)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
