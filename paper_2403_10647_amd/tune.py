"""Autotuner for the build's kernel knobs.

The knobs change how the work is cut, never what is computed: the radix digit
width (max_digit_bits: passes and digit widths of the sort), the tile shape of
the radix passes (sort_shape: workgroup size x items per thread), and whether
the first radix pass regenerates its keys from the expansion (fused_expand).
For a workload the tuner times every candidate setting (wall clock around
synchronized builds, launches included), checks that each one produces exactly
the grid of the default setting, and keeps the fastest.  Results are cached in a JSON file keyed by the device and a workload
signature (plain or batched, sort-key bits, order of magnitude of the pair
count), so later processes apply them without timing again.

    python -m paper_2403_10647_amd.tune --workload arch      # tune the 10M scene, print the table
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import time
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

KNOBS = ("max_digit_bits", "sort_shape", "fused_expand")
DEFAULTS = {"max_digit_bits": 9, "sort_shape": 3, "fused_expand": 0}
SPACE = {"max_digit_bits": (8, 9, 10, 11), "sort_shape": (0, 1, 2, 3, 4), "fused_expand": (0, 1)}


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "paper_2403_10647_amd", "tune.json")


def signature(batched: bool, key_bits: int, npairs: int) -> str:
    """Workloads that share this string share their best setting."""
    mag = 0 if npairs <= 0 else int(math.floor(math.log2(npairs)))
    return f"{'batched' if batched else 'plain'}:bits{key_bits}:pairs2^{mag}"


def candidates(space: Optional[Dict[str, Sequence[int]]] = None) -> List[Dict[str, int]]:
    sp = dict(SPACE)
    if space:
        sp.update(space)
    return [dict(zip(KNOBS, v)) for v in itertools.product(*(sp[k] for k in KNOBS))]


def load_cache(path: str) -> dict:
    try:
        with open(path) as fh:
            d = json.load(fh)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(path: str, cache: dict) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(cache: dict, device: str, sig: str) -> Optional[Dict[str, int]]:
    e = cache.get(device, {}).get(sig)
    if not e or not all(k in e.get("knobs", {}) for k in KNOBS):
        return None
    return {k: int(e["knobs"][k]) for k in KNOBS}


def record(cache: dict, device: str, sig: str, knobs: Dict[str, int], ms: float, table: list) -> dict:
    cache.setdefault(device, {})[sig] = {"knobs": dict(knobs), "ms": ms, "candidates": table}
    return cache


# ---- GPU side --------------------------------------------------------------------

def _set(G, knobs: Dict[str, int]) -> None:
    for k in KNOBS:
        G.tune_set(k, int(knobs[k]))


def set_knobs(G, knobs: Dict[str, int]) -> None:
    """Set every tuned knob (a setting from tune_plain, tune_batched or DEFAULTS)."""
    _set(G, knobs)


def confirm_plain(g, best: Dict[str, int], rounds: int = 3, reps: int = 10, G=None) -> Tuple[Dict[str, int], dict]:
    """Time ``best`` against the defaults in alternating rounds on plain builds of ``g``
    and keep the faster by median; returns (knobs, medians in ms)."""
    import statistics
    import torch
    if G is None:
        from . import _lib as G
    ws = G.Workspace()
    npairs, _ = G.count(g, ws)
    ws.get(max_workspace(G, g, npairs))
    out = G.build(g, cap_pairs=npairs, ws=ws)
    run = G.PlainBuild(g, out, ws)
    old = {k: G.tune_get(k) for k in KNOBS}
    times = {"default": [], "tuned": []}
    try:
        for _ in range(rounds):
            for name, knobs in (("default", DEFAULTS), ("tuned", best)):
                _set(G, knobs)
                run()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    run()
                torch.cuda.synchronize()
                times[name].append((time.perf_counter() - t0) * 1e3 / reps)
    finally:
        _set(G, old)
    med = {k: round(statistics.median(v), 5) for k, v in times.items()}
    return (dict(best) if med["tuned"] < med["default"] else dict(DEFAULTS)), med


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0)


def _key_bits(ncells: int) -> int:
    return max(1, (ncells - 1).bit_length())


def max_workspace(G, g, npairs: int, space=None) -> int:
    """Workspace bytes a plain build of ``g`` needs under the widest-sized of the
    candidate digit widths (a wider digit keeps more look-back words per tile)."""
    sp = dict(SPACE)
    if space:
        sp.update(space)
    old = G.tune_get("max_digit_bits")
    try:
        need = 0
        for d in sp["max_digit_bits"]:
            G.tune_set("max_digit_bits", int(d))
            need = max(need, G.workspace_size(g.ntris, npairs, g.res))
    finally:
        G.tune_set("max_digit_bits", old)
    return need


def tune_plain(g, reps: int = 5, space=None, cache_path: Optional[str] = None, G=None) -> Tuple[Dict[str, int], list]:
    """Best setting for plain builds of ``g`` (a GridInput); returns (knobs, table)."""
    import torch
    if G is None:
        from . import _lib as G
    ws = G.Workspace()
    npairs, _ = G.count(g, ws)
    ws.get(max_workspace(G, g, npairs, space))   # sized once for every candidate: PlainBuild keeps its pointer
    out = G.build(g, cap_pairs=npairs, ws=ws)
    run = G.PlainBuild(g, out, ws)

    def snapshot():
        return [t.clone() for t in (out.cells[:out.npairs], out.objs[:out.npairs], out.ranges)]

    best, table = _search(G, run, snapshot, reps, space)
    if cache_path:
        sig = signature(False, _key_bits(g.ncells), npairs)
        save_cache(cache_path, record(load_cache(cache_path), _device_name(), sig, best, table[0]["ms"], table))
    return best, table


def tune_batched(inputs, reps: int = 3, space=None, cache_path: Optional[str] = None, G=None):
    """Best setting for batched builds of ``inputs`` (GridInputs); returns (knobs, table)."""
    if G is None:
        from . import _lib as G
    ws = G.Workspace()
    caps = G.count_batched(inputs, ws)
    outs = G.alloc_results(inputs, caps)

    def run():
        return G.build_batched(inputs, outs, ws)

    def snapshot():
        return [t.clone() for o in outs for t in (o.cells[:o.npairs], o.objs[:o.npairs], o.ranges)]

    best, table = _search(G, run, snapshot, reps, space)
    if cache_path:
        sig = signature(True, _key_bits(sum(g.ncells for g in inputs)), sum(caps))
        save_cache(cache_path, record(load_cache(cache_path), _device_name(), sig, best, table[0]["ms"], table))
    return best, table


def _search(G, run, snapshot, reps, space):
    import torch
    old = {k: G.tune_get(k) for k in KNOBS}
    table = []
    try:
        _set(G, DEFAULTS)
        run()
        torch.cuda.synchronize()
        ref = snapshot()
        for knobs in candidates(space):
            _set(G, knobs)
            run()                                   # warm-up (and first-use costs)
            torch.cuda.synchronize()
            same = all(torch.equal(a, b) for a, b in zip(ref, snapshot()))
            t0 = time.perf_counter()
            for _ in range(reps):
                run()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / reps   # what a caller waits for, launches included
            table.append({"knobs": knobs, "ms": round(ms, 5), "identical": bool(same)})
    finally:
        _set(G, old)
    bad = [r for r in table if not r["identical"]]
    if bad:
        # a knob may change how the work is cut, never the grid
        raise RuntimeError(f"settings changed the grid: {[r['knobs'] for r in bad]}")
    table.sort(key=lambda r: r["ms"])
    return dict(table[0]["knobs"]), table


def apply(batched: bool, key_bits: int, npairs: int, cache_path: Optional[str] = None, G=None) -> Optional[Dict[str, int]]:
    """Set the cached best knobs for this workload, if any; returns them."""
    if G is None:
        from . import _lib as G
    path = cache_path or default_cache_path()
    knobs = lookup(load_cache(path), _device_name(), signature(batched, key_bits, npairs))
    if knobs:
        _set(G, knobs)
    return knobs


def main(argv: Optional[Iterable[str]] = None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="arch", choices=["arch", "mixed", "small", "batch"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--cache", default=default_cache_path())
    ap.add_argument("--ngrids", type=int, default=512)
    args = ap.parse_args(list(argv) if argv is not None else None)
    from . import _lib as G
    from . import scenes
    G.lib()
    if args.workload == "batch":
        inputs = [G.GridInput.from_scene(s) for s in scenes.make_batch(args.seed, ngrids=args.ngrids)]
        best, table = tune_batched(inputs, args.reps, cache_path=args.cache, G=G)
    else:
        g = G.GridInput.from_scene(scenes.make_scene(args.workload, seed=args.seed))
        best, table = tune_plain(g, args.reps, cache_path=args.cache, G=G)
    print(json.dumps({"workload": args.workload, "best": best, "cache": args.cache,
                      "table": table[:10]}), flush=True)


if __name__ == "__main__":
    main()
