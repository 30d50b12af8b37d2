"""Continuous-batching server for grid builds.

Requests (a scene each, already in device memory) arrive over time.  On
arrival a request is counted (CountCells + ExclusiveSum, Algorithm 1), which
predicts its pair count NO exactly; from NO and the cell count R follow the
bytes its outputs need, and the request is admitted when they fit in the
device-memory budget next to the resident workspaces.  Admitted requests wait
in a FIFO queue; whenever a slot (a stream with its own resident workspace and
pinned staging) is free, the requests at the head of the queue are built
together as one batched build with no host synchronisation.  Several slots
are in flight at once, so requests that arrive while others are on the GPU
overlap with them on the device.  When a slot's completion event has passed,
its requests are complete: their latency runs from the scheduled arrival to
the moment the host observes the completion.

Every output can be compared on the device with a reference output of the same
scene (its stand-alone build); mismatches are counted per slot and read back
once at the end, off the timed path.

Batch formation (``form_batch``) is pure host logic: FIFO order, a cap on
grids and pairs per batch, the batch's cells within one 32-bit key space, and
the byte budget.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib as G


MAX_BATCH_CELLS = 1 << 32   # a batch numbers its grids' cells in one 32-bit key space


def bits_for(n: int) -> int:
    """Bits needed to hold the values 0..n-1."""
    return 0 if n <= 1 else int(n - 1).bit_length()


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds after the start of the run
    inp: G.GridInput
    key: int = -1                  # index of the reference output to check against (-1: none)
    npairs: int = -1               # predicted by the count at arrival
    out_bytes: int = 0
    done: float = -1.0
    status: int = 0                # GRID_OK, or why the request failed / was rejected
    result: Optional[G.GridResult] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def output_bytes(npairs: int, ncells: int) -> int:
    """Device bytes of one request's outputs: cells and objs (4 B per pair each), ranges (8 B per cell)."""
    return 8 * max(npairs, 1) + 8 * ncells


def batch_workspace_bytes(inputs: Sequence[G.GridInput], caps: Sequence[int]) -> int:
    """Workspace bytes of one batched build of ``inputs`` with pair capacities ``caps``."""
    arr = G._descs(list(inputs))
    for d, c in zip(arr, caps):
        d.out.cap_pairs = int(c)
    return int(G.lib().grid_workspace_size_batched(arr, len(inputs)))


def form_batch(queue: Sequence[Request], free_bytes: int, max_grids: int, max_pairs: int) -> int:
    """How many requests from the head of the FIFO queue go into the next batch.

    The batch grows while the next request's outputs fit in free_bytes, the
    batch's cells (all grids numbered in one space) still fit 32-bit sort keys,
    the batch holds at most max_grids grids and, unless it is empty, at most
    max_pairs pairs.  Returns 0 when the head itself does not fit in free_bytes."""
    n = 0
    used = 0
    pairs = 0
    cells = 0
    for r in queue:
        if n >= max_grids:
            break
        if cells + r.inp.ncells > MAX_BATCH_CELLS:
            break
        if n > 0 and pairs + r.npairs > max_pairs:
            break
        if used + r.out_bytes > free_bytes:
            break
        n += 1
        used += r.out_bytes
        pairs += r.npairs
        cells += r.inp.ncells
    return n


class _Slot:
    def __init__(self, device, ws_bytes: int, max_grids: int):
        self.stream = torch.cuda.Stream(device=device)
        self.ws = G.Workspace(device)
        self.ws.get(ws_bytes)
        self.ws_bytes = ws_bytes
        self.staging = torch.empty(int(G.lib().grid_batch_staging_size(max_grids)), dtype=torch.uint8,
                                   pin_memory=True)
        self.event = torch.cuda.Event()
        self.batch: List[Request] = []
        self.bytes = 0
        self.arena = None
        self.mismatch = torch.zeros((), dtype=torch.int64, device=device)


@dataclasses.dataclass
class ServeStats:
    requests: int
    completed: int
    rejected: int
    failed: int
    duration_s: float
    builds_per_s: float
    pairs_per_s: float
    p50_ms: float
    p99_ms: float
    max_ms: float
    batches: int
    mean_batch: float
    peak_bytes: int
    budget_bytes: int
    verified: int
    mismatches: int
    peak_slots: int = 0            # most batches on the device at one time

    def as_dict(self):
        return dataclasses.asdict(self)


class Server:
    """One device, ``nslots`` batches in flight, admission against ``budget_bytes``.

    ``ws_bytes`` is each slot's resident workspace; the budget covers the
    workspaces and the outputs of every admitted request until it completes."""

    def __init__(self, budget_bytes: int, ws_bytes: int, nslots: int = 3, max_grids: int = 512,
                 max_pairs: int = 1 << 25, references: Optional[Sequence[G.GridResult]] = None,
                 keep_results: bool = False, device=None):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.budget = int(budget_bytes)
        self.ws_bytes = int(ws_bytes)
        if self.ws_bytes * nslots >= self.budget:
            raise ValueError("the slot workspaces alone exceed the budget")
        self.max_grids = max_grids
        self.max_pairs = max_pairs
        self.refs = references
        self.keep = keep_results
        self.slots = [_Slot(self.device, self.ws_bytes, max_grids) for _ in range(nslots)]
        self.count_stream = torch.cuda.Stream(device=self.device)
        self.count_ws = G.Workspace(self.device)
        self.out_budget = self.budget - self.ws_bytes * nslots

    # -- admission count -----------------------------------------------------
    def _count(self, new: List[Request]) -> List[int]:
        """Pair counts of newly arrived requests, counted together; if that fails, one
        by one, so a bad request fails alone (its entry is then its negative status)."""
        try:
            return G.count_batched([r.inp for r in new], self.count_ws, self.count_stream)
        except G.GridError:
            pass
        out = []
        for r in new:
            try:
                out.append(G.count_batched([r.inp], self.count_ws, self.count_stream)[0])
            except G.GridError as e:
                out.append(e.status)
        return out

    # -- one batch ---------------------------------------------------------
    def _launch(self, slot: _Slot, batch: List[Request]) -> List[Request]:
        """Launch ``batch`` on ``slot``; returns the requests that could not be launched."""
        inputs = [r.inp for r in batch]
        while True:
            caps = [r.npairs for r in batch]
            with torch.cuda.stream(slot.stream):
                tot_pairs = sum(max(c, 1) for c in caps)
                tot_ranges = sum(2 * g.ncells for g in inputs)
                cells = torch.empty(tot_pairs, dtype=torch.int32, device=self.device)
                objs = torch.empty(tot_pairs, dtype=torch.int32, device=self.device)
                ranges = torch.empty(tot_ranges, dtype=torch.int32, device=self.device)
            outs = []
            p = q = 0
            for g, c in zip(inputs, caps):
                n = max(c, 1)
                outs.append(G.GridResult(cells[p:p + n], objs[p:p + n], ranges[q:q + 2 * g.ncells], 0))
                p += n
                q += 2 * g.ncells
            arr = G._descs(inputs, outs)
            need = int(G.lib().grid_workspace_size_batched(arr, len(inputs)))
            if need <= slot.ws_bytes or len(batch) == 1:
                break
            batch, inputs = batch[:-1], inputs[:-1]
        if need > slot.ws_bytes:
            batch[0].status = G.GRID_E_NOMEM
            return []
        st = G.lib().grid_build_batched_async(arr, len(inputs), G.C.c_void_p(slot.ws.buf.data_ptr()),
                                              G.C.c_size_t(slot.ws_bytes), G.C.c_void_p(slot.staging.data_ptr()),
                                              G.C.c_size_t(slot.staging.numel()), G.C.c_void_p(slot.stream.cuda_stream))
        if st != G.GRID_OK:
            for r in batch:
                r.status = st
            return []
        slot.event.record(slot.stream)
        if self.refs is not None:
            self._verify(slot, batch, outs, cells, objs, ranges)
        for r, o, c in zip(batch, outs, caps):
            o.npairs = c
            r.result = o
        slot.batch = batch
        slot.arena = (cells, objs, ranges)
        slot.bytes = sum(r.out_bytes for r in batch)
        return []

    def _verify(self, slot, batch, outs, cells, objs, ranges):
        with torch.cuda.stream(slot.stream):
            rc, ro, rr = [], [], []
            for r, o in zip(batch, outs):
                ref = self.refs[r.key]
                n = max(r.npairs, 1)
                if r.npairs == 0:
                    # the empty slot of an empty grid holds no output: compare it with itself
                    rc.append(o.cells)
                    ro.append(o.objs)
                else:
                    rc.append(ref.cells[:n])
                    ro.append(ref.objs[:n])
                rr.append(ref.ranges)
            slot.mismatch += (cells != torch.cat(rc)).sum() + (objs != torch.cat(ro)).sum() + \
                (ranges != torch.cat(rr)).sum()

    def _finish(self, slot: _Slot, now: float):
        st, _ = G.workspace_status(slot.ws, slot.stream)
        for r in slot.batch:
            r.done = now
            r.status = st
            if not self.keep:
                r.result = None
        slot.batch = []
        slot.arena = None
        freed = slot.bytes
        slot.bytes = 0
        return freed

    # -- the loop ----------------------------------------------------------
    def run(self, requests: Sequence[Request], clock: Callable[[], float] = time.perf_counter) -> ServeStats:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        n = len(reqs)
        for s in self.slots:
            s.mismatch.zero_()
        torch.cuda.synchronize(self.device)
        queue: List[Request] = []
        used = 0
        peak = 0
        peak_slots = 0
        nxt = 0
        finished = 0
        batches = 0
        batched = 0
        t0 = clock()
        while finished < n:
            now = clock() - t0
            # arrivals: count them together, on their own stream
            j = nxt
            while j < n and reqs[j].arrival <= now:
                j += 1
            if j > nxt:
                new = reqs[nxt:j]
                nxt = j
                caps = self._count(new)
                for k, r in enumerate(new):
                    if caps[k] < 0:            # this request's own count failed (e.g. a bad vertex index)
                        r.status = caps[k]
                        r.done = clock() - t0
                        finished += 1
                        continue
                    r.npairs = caps[k]
                    r.out_bytes = output_bytes(r.npairs, r.inp.ncells)
                    if r.out_bytes > self.out_budget:
                        r.status = G.GRID_E_NOMEM
                        r.done = clock() - t0
                        finished += 1
                    else:
                        queue.append(r)
            # completions
            for s in self.slots:
                if s.batch and s.event.query():
                    k = len(s.batch)
                    used -= self._finish(s, clock() - t0)
                    finished += k
            # launches
            for s in self.slots:
                if s.batch or not queue:
                    continue
                k = form_batch(queue, self.out_budget - used, self.max_grids, self.max_pairs)
                if k == 0:
                    break
                batch = queue[:k]
                self._launch(s, batch)
                launched = len(s.batch)
                if launched == 0:
                    # the head could not be built (too large for a workspace, or an error)
                    r = queue.pop(0)
                    r.done = clock() - t0
                    finished += 1
                    continue
                del queue[:launched]
                used += s.bytes
                peak = max(peak, used)
                peak_slots = max(peak_slots, sum(1 for x in self.slots if x.batch))
                batches += 1
                batched += launched
            if not queue and all(not s.batch for s in self.slots) and nxt < n:
                wait = reqs[nxt].arrival - (clock() - t0)
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
        t_end = clock() - t0
        torch.cuda.synchronize(self.device)
        mism = int(sum(int(s.mismatch.item()) for s in self.slots)) if self.refs is not None else 0
        ok = [r for r in reqs if r.status == G.GRID_OK]
        rej = [r for r in reqs if r.status == G.GRID_E_NOMEM]
        lat = np.asarray([r.latency for r in ok]) * 1e3 if ok else np.zeros(1)
        first = reqs[0].arrival if reqs else 0.0
        last = max((r.done for r in ok), default=t_end)
        span = max(last - first, 1e-9)
        return ServeStats(
            requests=n, completed=len(ok), rejected=len(rej), failed=n - len(ok) - len(rej),
            duration_s=t_end, builds_per_s=len(ok) / span, pairs_per_s=sum(r.npairs for r in ok) / span,
            p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)), max_ms=float(lat.max()),
            batches=batches, mean_batch=batched / max(batches, 1), peak_bytes=peak, budget_bytes=self.budget,
            verified=len(ok) if self.refs is not None else 0, mismatches=mism, peak_slots=peak_slots)


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process of ``rate`` per second over [0, duration)."""
    rng = np.random.default_rng(np.random.SeedSequence(entropy=seed, spawn_key=(4, 1)))
    n = int(rate * duration * 1.2 + 10 * math.sqrt(rate * duration + 1) + 16)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    while t[-1] < duration:
        t = np.concatenate([t, t[-1] + np.cumsum(rng.exponential(1.0 / rate, size=n))])
    return t[t < duration]


def make_requests(pool: Sequence[G.GridInput], rate: float, duration: float, seed: int,
                  big: Optional[G.GridInput] = None, big_every: float = 1.0, big_key: int = -1,
                  burst: bool = False) -> List[Request]:
    """Requests drawn uniformly from ``pool`` at Poisson times (all at t = 0 when ``burst``), plus the
    ``big`` scene at t = 0, big_every, 2 big_every, ...  Request keys index the pool (the big scene
    takes ``big_key``)."""
    times = poisson_arrivals(rate, duration, seed)
    rng = np.random.default_rng(np.random.SeedSequence(entropy=seed, spawn_key=(4, 2)))
    keys = rng.integers(0, len(pool), size=len(times))
    reqs = [Request(i, 0.0 if burst else float(t), pool[int(k)], int(k)) for i, (t, k) in enumerate(zip(times, keys))]
    if big is not None:
        m = len(reqs)
        nb = int(math.ceil(duration / big_every))
        reqs += [Request(m + b, 0.0 if burst else b * big_every, big, big_key) for b in range(nb)]
    return reqs


def plain_builds_per_s(requests: Sequence[Request], ws: Optional[G.Workspace] = None) -> Dict[str, float]:
    """The same requests built one at a time with grid_build (count, readback, build), for comparison."""
    ws = ws or G.Workspace()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pairs = 0
    for r in requests:
        res = G.build(r.inp, ws=ws)
        pairs += res.npairs
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"builds_per_s": len(requests) / dt, "pairs_per_s": pairs / dt, "seconds": dt}
