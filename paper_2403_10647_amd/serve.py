"""Continuous-batching server for grid builds.

Requests (a scene each, already in device memory) arrive over time.  Whenever
a slot (a stream with its own resident workspace and pinned staging) is free,
the requests that have arrived are counted there together (CountCells +
ExclusiveSum, Algorithm 1) without a host wait.  The count predicts each
request's pair count NO exactly; from NO and the cell count R follow the bytes
its outputs need.  When the slot's count has completed and those bytes fit in
the device-memory budget next to the resident workspaces, the outputs are
allocated and the same build resumes from its count (radix passes and ranges
only), again without a host wait.  A request larger than the whole budget is
rejected.  Several slots are in flight at once, so requests that arrive while
others are on the GPU overlap with them on the device.  When a slot's
completion event has passed, its requests are complete: their latency runs from
the scheduled arrival to the moment the host observes the completion.

Counted batches that cannot resume (a bad request among them, more pairs than
the slot's workspace holds, outputs above the budget) fall back to a FIFO
queue of counted requests, built as whole batched builds (count included)
that form_batch sizes to the budget, the pair cap and the workspace.

Every output can be compared on the device with a reference output of the same
scene (its stand-alone build); mismatches are counted per slot and read back
once at the end, off the timed path.

Batch formation (``form_batch``, ``form_count_batch``) is pure host logic: FIFO
order, a cap on grids (and pairs) per batch, the batch's cells within one
32-bit key space, and the byte budget.
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


def form_count_batch(arrived: Sequence[Request], max_grids: int, max_pairs: int, pairs_per_tri: float) -> int:
    """How many requests from the head of the arrival FIFO are counted together (at least one):
    at most max_grids, their cells within one 32-bit key space, and, unless the batch is empty,
    at most max_pairs pairs predicted at pairs_per_tri pairs per triangle (NO is only known
    after the count)."""
    n = 0
    cells = 0
    pairs = 0.0
    for r in arrived:
        p = r.inp.ntris * pairs_per_tri
        if n > 0 and (n >= max_grids or cells + r.inp.ncells > MAX_BATCH_CELLS or pairs + p > max_pairs):
            break
        n += 1
        cells += r.inp.ncells
        pairs += p
    return n


class _Slot:
    def __init__(self, device, ws_bytes: int, max_grids: int):
        self.stream = torch.cuda.Stream(device=device)
        self.ws = G.Workspace(device)
        self.ws.get(ws_bytes)
        self.ws_bytes = ws_bytes
        # two tables: the counted one stays while the resumed build copies the second
        self.staging = torch.empty(2 * int(G.lib().grid_batch_staging_size(max_grids)), dtype=torch.uint8,
                                   pin_memory=True)
        self.counts = torch.zeros(max_grids + 1, dtype=torch.int64, pin_memory=True)
        self.counted = torch.cuda.Event()
        self.counting: List[Request] = []    # requests counted on this slot, not yet built
        self.event = torch.cuda.Event()
        self.batch: List[Request] = []
        self.bytes = 0
        self.arena = None
        self.pair_at: List[int] = []         # each request's first pair in the arena
        self.descs = None                    # descriptor array of the counted batch
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
        # pairs per triangle seen so far (sizes count batches before their NO is known)
        self.seen_tris = 0
        self.seen_pairs = 0

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

    # -- outputs -----------------------------------------------------------
    def _outputs(self, slot: _Slot, inputs: List[G.GridInput], caps: List[int]):
        """One device allocation (on the slot's stream) holding every grid's cells, objs and ranges:
        (arena (cells, objs, ranges), each grid's first pair and first range word)."""
        tot_pairs = sum(max(c, 1) for c in caps)
        tot_ranges = sum(2 * g.ncells for g in inputs)
        with torch.cuda.stream(slot.stream):
            buf = torch.empty(2 * tot_pairs + tot_ranges, dtype=torch.int32, device=self.device)
        arena = (buf[:tot_pairs], buf[tot_pairs:2 * tot_pairs], buf[2 * tot_pairs:])
        pair_at, range_at = [], []
        p = q = 0
        for g, c in zip(inputs, caps):
            pair_at.append(p)
            range_at.append(q)
            p += max(c, 1)
            q += 2 * g.ncells
        return arena, pair_at, range_at

    def _out_descs(self, arr, inputs, caps, arena, pair_at, range_at):
        """Write the outputs' addresses into the descriptor array ``arr``."""
        c0, o0, r0 = (x.data_ptr() for x in arena)
        G._set_outputs(arr, [c0 + 4 * p for p in pair_at], [o0 + 4 * p for p in pair_at],
                       [r0 + 4 * q for q in range_at], [max(c, 1) for c in caps])

    def _started(self, slot: _Slot, batch: List[Request], arena, pair_at, range_at):
        slot.event.record(slot.stream)
        cells, objs, ranges = arena
        for r, p, q in zip(batch, pair_at, range_at):
            if self.keep:
                n = max(r.npairs, 1)
                r.result = G.GridResult(cells[p:p + n], objs[p:p + n], ranges[q:q + 2 * r.inp.ncells], r.npairs)
        slot.batch = batch
        slot.arena = arena
        slot.pair_at = pair_at
        slot.bytes = sum(r.out_bytes for r in batch)

    # -- a batch counted on its slot, then resumed ---------------------------
    def _count_on(self, slot: _Slot, batch: List[Request]) -> bool:
        """Enqueue the count of ``batch`` on ``slot``; False if the workspace cannot hold even the count."""
        inputs = [r.inp for r in batch]
        arr = G._descs(inputs)
        try:
            G.count_batched_async(inputs, slot.ws, slot.ws_bytes, slot.staging, slot.counts, slot.stream, descs=arr)
        except G.GridError:
            return False
        slot.counted.record(slot.stream)
        slot.counting = batch
        slot.descs = arr
        return True

    def _resume(self, slot: _Slot, free_bytes: int):
        """Admission of the batch counted on ``slot`` once its count has completed.

        Returns (state, requests): "built" (the build resumed on the slot), "wait" (its outputs do not
        fit in free_bytes yet), "failed" (the resumed build was refused: the requests carry its
        status), or "fallback" (the requests are handed back, counted where possible, for the
        whole-batch path; their npairs is set, or their status if their own count failed)."""
        batch = slot.counting
        k = len(batch)
        c = slot.counts[:k + 1].tolist()
        status = c[k]
        if status & (G.COUNT_BAD_INDEX | G.COUNT_INTERNAL | G.COUNT_OVER_32BIT):
            # a bad request among them, or 32-bit pair starts that wrapped: counted again one by
            # one, so that a bad request fails alone
            slot.counting = []
            for r, n in zip(batch, self._count(batch)):
                if n < 0:
                    r.status = n
                else:
                    r.npairs = n
                    r.out_bytes = output_bytes(n, r.inp.ncells)
            return "fallback", batch
        for r, n in zip(batch, c[:k]):
            r.npairs = int(n)
            r.out_bytes = output_bytes(r.npairs, r.inp.ncells)
            self.seen_tris += r.inp.ntris
            self.seen_pairs += r.npairs
        need = sum(r.out_bytes for r in batch)
        if status or need > self.out_budget:
            slot.counting = []
            return "fallback", batch
        if need > free_bytes:
            return "wait", []
        slot.counting = []
        inputs = [r.inp for r in batch]
        caps = c[:k]
        arena, pair_at, range_at = self._outputs(slot, inputs, caps)
        self._out_descs(slot.descs, inputs, caps, arena, pair_at, range_at)
        try:
            G.build_batched_counted(inputs, None, caps, slot.ws, slot.ws_bytes, slot.staging, slot.stream,
                                    descs=slot.descs)
        except G.GridError as e:
            for r in batch:
                r.status = e.status
            return "failed", batch
        self._started(slot, batch, arena, pair_at, range_at)
        return "built", batch

    # -- one whole batch (count included) --------------------------------------
    def _launch(self, slot: _Slot, batch: List[Request]) -> List[Request]:
        """Launch ``batch`` on ``slot``; returns the requests that could not be launched."""
        inputs = [r.inp for r in batch]
        while True:
            caps = [r.npairs for r in batch]
            arena, pair_at, range_at = self._outputs(slot, inputs, caps)
            arr = G._descs(inputs)
            self._out_descs(arr, inputs, caps, arena, pair_at, range_at)
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
        self._started(slot, batch, arena, pair_at, range_at)
        return []

    def _verify(self, slot: _Slot):
        """Compare the slot's outputs with the references on the device (queued after the build on the
        slot's stream, once its requests are complete, so that it adds to no request's latency)."""
        cells, objs, ranges = slot.arena
        with torch.cuda.stream(slot.stream):
            rc, ro, rr = [], [], []
            for r, p in zip(slot.batch, slot.pair_at):
                ref = self.refs[r.key]
                if r.npairs == 0:
                    # the one-pair slot of an empty grid holds no output: compare it with itself
                    rc.append(cells[p:p + 1])
                    ro.append(objs[p:p + 1])
                else:
                    rc.append(ref.cells[:r.npairs])
                    ro.append(ref.objs[:r.npairs])
                rr.append(ref.ranges)
            slot.mismatch += (cells != torch.cat(rc)).sum() + (objs != torch.cat(ro)).sum() + \
                (ranges != torch.cat(rr)).sum()

    def _finish(self, slot: _Slot, now: float):
        st, _ = G.workspace_status(slot.ws, slot.stream)
        for r in slot.batch:
            r.done = now
            r.status = st
        if self.refs is not None and st == G.GRID_OK:
            self._verify(slot)
        if not self.keep:
            for r in slot.batch:
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
        arrived: List[Request] = []    # not yet counted, FIFO
        queue: List[Request] = []      # counted, for whole batched builds, FIFO
        counted: List[_Slot] = []      # slots holding a counted batch, in count order
        used = 0
        peak = 0
        peak_slots = 0
        nxt = 0
        finished = 0
        batches = 0
        batched = 0
        t0 = clock()

        def settle(r: Request) -> int:
            """A counted request from a failed resume: queued, or finished (failed or above the budget)."""
            if r.status != G.GRID_OK:
                r.done = clock() - t0
                return 1
            if r.out_bytes > self.out_budget:
                r.status = G.GRID_E_NOMEM
                r.done = clock() - t0
                return 1
            queue.append(r)
            return 0

        while finished < n:
            now = clock() - t0
            while nxt < n and reqs[nxt].arrival <= now:
                arrived.append(reqs[nxt])
                nxt += 1
            # completions
            for s in self.slots:
                if s.batch and s.event.query():
                    k = len(s.batch)
                    used -= self._finish(s, clock() - t0)
                    finished += k
            # counted batches, in count order: resume when their outputs fit
            while counted and counted[0].counted.query():
                s = counted[0]
                state, batch = self._resume(s, self.out_budget - used)
                if state == "wait":
                    break
                counted.pop(0)
                if state == "built":
                    used += s.bytes
                    peak = max(peak, used)
                    peak_slots = max(peak_slots, sum(1 for x in self.slots if x.batch))
                    batches += 1
                    batched += len(batch)
                elif state == "failed":
                    for r in batch:
                        r.done = clock() - t0
                    finished += len(batch)
                else:
                    finished += sum(settle(r) for r in batch)
            # whole batched builds of the requests handed back, then counts of new arrivals
            for s in self.slots:
                if s.batch or s.counting:
                    continue
                if queue:
                    k = form_batch(queue, self.out_budget - used, self.max_grids, self.max_pairs)
                    if k == 0:
                        continue
                    self._launch(s, queue[:k])
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
                elif arrived:
                    ppt = 1.25 * self.seen_pairs / self.seen_tris if self.seen_tris else 16.0
                    k = form_count_batch(arrived, self.max_grids, self.max_pairs, ppt)
                    batch = arrived[:k]
                    del arrived[:k]
                    if self._count_on(s, batch):
                        counted.append(s)
                    else:
                        # the workspace cannot hold even their count: counted apart, built whole
                        for r, c in zip(batch, self._count(batch)):
                            if c < 0:
                                r.status = c
                            else:
                                r.npairs = c
                                r.out_bytes = output_bytes(c, r.inp.ncells)
                        finished += sum(settle(r) for r in batch)
            idle = not arrived and not queue and not counted and all(not s.batch for s in self.slots)
            if idle and nxt < n:
                # sleep until a millisecond before the next arrival (sleeps overshoot), then poll
                wait = reqs[nxt].arrival - (clock() - t0)
                if wait > 2e-3:
                    time.sleep(wait - 1e-3)
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


def spaced_requests(pool: Sequence[G.GridInput], gap: float, count: int, seed: int) -> List[Request]:
    """``count`` requests drawn uniformly from ``pool``, one every ``gap`` seconds (request keys index the pool)."""
    rng = np.random.default_rng(np.random.SeedSequence(entropy=seed, spawn_key=(4, 3)))
    keys = rng.integers(0, len(pool), size=count)
    return [Request(i, i * gap, pool[int(k)], int(k)) for i, k in enumerate(keys)]


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
