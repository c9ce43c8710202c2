"""Continuous-batching serving loop for the transient NLOS forward operator.

Requests (a depth map with its albedo and mask, plus system parameters)
arrive over time.  Each tick admits waiting requests in arrival order while
their device footprint fits in an HBM budget. It then uploads their maps,
builds all their patch records with one batched geometry call and runs all
their forward models with one batched forward call (the K-frame loop of
Algorithm 1, many scenes at once).  Records and histograms stay on the
device; a request's memory is returned to the budget when its tick's
completion event has passed.  Up to ``depth`` ticks are in flight, so the
host prepares the next tick while the GPU runs the current one.

``mode="plain"`` serves the same stream one request per tick through the
single-request calls: the baseline that batching is measured against.
Every request computes exactly what it computes alone.

Latency of a request = completion of its tick on the GPU (an event timed
against a start event recorded when serving begins) minus its arrival time.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import (Batcher, forward, forward_batched, n_histograms, params_of, patches_batched,
               patches_from_depth)
from ._native import NLOS_RECORD_FLOATS

RECORD_BYTES = 4 * NLOS_RECORD_FLOATS
STAT_BYTES_PER_RECORD = 32.0 / 256.0   # one 32-byte summary per 256 records


def footprint_bytes(req) -> int:
    """Device bytes a request holds while in flight: its maps, its patch
    records, its output histograms and its workspace share."""
    g = req.patch_grid
    npx = int(g["nx"]) * int(g["ny"])
    maps = 4 * npx + (4 * npx if req.albedo is not None else 0) + (npx if req.mask is not None else 0)
    rec = RECORD_BYTES * npx + 4
    out = 4 * n_histograms(params_of(req)) * int(req.n_bins)
    ws = int(STAT_BYTES_PER_RECORD * npx) + 2048 + 8 * (npx // 1024 + 1)
    return maps + rec + out + ws


def pair_count(req) -> int:
    """Histogram x present-patch pairs of a request (its work), counted on
    the host maps with the presence rule of the geometry kernel."""
    present = np.isfinite(req.depth) & (req.depth > 0)
    if req.albedo is not None:
        present &= req.albedo > 0
    if req.mask is not None:
        present &= req.mask != 0
    return int(n_histograms(params_of(req))) * int(present.sum())


class Admission:
    """First-come first-served admission under a byte budget: a tick takes
    waiting requests in arrival order until the next one would overflow the
    budget or the tick is full (no overtaking, so no request starves).  A
    request larger than the whole budget is rejected when it reaches the head
    of the queue."""

    def __init__(self, budget_bytes: int, max_batch: int):
        if budget_bytes <= 0 or max_batch <= 0:
            raise ValueError("budget and batch size must be positive")
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.in_use = 0
        self.peak = 0

    def admit(self, queue: collections.deque, sizes: Sequence[int], work: Optional[Sequence[float]] = None,
              max_work: float = float("inf")):
        """Pop admitted request ids from the head of ``queue``; returns
        (admitted, rejected).  With ``work`` given, a tick also stops once its
        work reaches ``max_work`` (its first request is always taken)."""
        admitted, rejected = [], []
        w = 0.0
        while queue and len(admitted) < self.max_batch:
            i = queue[0]
            b = int(sizes[i])
            if b > self.budget:
                queue.popleft()
                rejected.append(i)
                continue
            if self.in_use + b > self.budget:
                break
            if work is not None and admitted and w + float(work[i]) > max_work:
                break
            queue.popleft()
            self.in_use += b
            admitted.append(i)
            if work is not None:
                w += float(work[i])
        self.peak = max(self.peak, self.in_use)
        return admitted, rejected

    def release(self, nbytes: int) -> None:
        self.in_use -= int(nbytes)
        if self.in_use < 0:
            raise RuntimeError("admission accounting went negative")


@dataclasses.dataclass
class ServeResult:
    latency_ms: np.ndarray        # per request (nan for rejected)
    done_ms: np.ndarray           # completion time since serving began
    makespan_ms: float
    ticks: int
    batch_sizes: List[int]
    peak_bytes: int
    rejected: List[int]
    outputs: Optional[list]       # per request device outputs (keep_outputs=True)

    def percentile(self, q: float) -> float:
        v = self.latency_ms[np.isfinite(self.latency_ms)]
        return float(np.percentile(v, q)) if v.size else float("nan")


class _Tick:
    __slots__ = ("ids", "event", "held", "bytes")

    def __init__(self, ids, event, held, nbytes):
        self.ids = ids
        self.event = event
        self.held = held
        self.bytes = nbytes


class Server:
    """One GPU, one stream, continuous batching under an HBM budget.

    budget_bytes    device bytes of the requests in flight (footprint_bytes).
    max_batch       requests per tick.
    depth           ticks in flight.
    max_tick_pairs  work per tick (pairs; the first request of a tick is
                    always taken): short ticks let requests complete soon
                    after their own work instead of at the end of a long
                    tick.  The default is a few milliseconds of GPU work.
    A tick of one request runs through the single-request calls (nothing to
    batch, so no table upload)."""

    def __init__(self, budget_bytes: int = 2 << 30, max_batch: int = 32, depth: int = 2,
                 mode: str = "batched", device="cuda", max_tick_pairs: float = 8e9):
        if mode not in ("batched", "plain"):
            raise ValueError("mode is 'batched' or 'plain'")
        self.max_tick_pairs = float(max_tick_pairs)
        self.budget = int(budget_bytes)
        self.max_batch = 1 if mode == "plain" else int(max_batch)
        self.depth = max(1, int(depth))
        self.mode = mode
        self.device = torch.device(device)
        # two batched calls per tick: enough pinned tables that a table is
        # only reused once its tick has left the pipeline
        self.batcher = Batcher(self.device, n_tables=2 * self.depth + 2)

    @staticmethod
    def stage(req):
        """Host payload of a request in pinned memory (done as a request is
        received, before it is queued)."""
        pin = lambda a, dt: None if a is None else torch.from_numpy(np.ascontiguousarray(a, dt)).pin_memory()
        return (pin(req.depth, np.float32), pin(req.albedo, np.float32), pin(req.mask, np.uint8))

    def _launch(self, reqs, staged, ids, stream):
        dev = self.device
        maps = []
        for i in ids:
            r = reqs[i]
            d, a, m = staged[i]
            depth = d.to(dev, non_blocking=True)
            albedo = None if a is None else a.to(dev, non_blocking=True)
            mask = None if m is None else m.to(dev, non_blocking=True)
            maps.append(dict(depth=depth, albedo=albedo, mask=mask, grid=r.patch_grid,
                             cosines=getattr(r, "cosines", True)))
        if self.mode == "batched" and len(ids) > 1:
            recs = patches_batched(maps, batcher=self.batcher, stream=stream)
            outs = forward_batched([(params_of(reqs[i]), p, n, None) for i, (p, n) in zip(ids, recs)],
                                   batcher=self.batcher, stream=stream)
        else:
            recs, outs = [], []
            for i, mp in zip(ids, maps):
                p, n = patches_from_depth(mp["depth"], mp["grid"], mp["albedo"], mp["mask"],
                                          cosines=mp["cosines"], stream=stream)
                outs.append(forward(params_of(reqs[i]), p, n, stream=stream))
                recs.append((p, n))
        return outs, (maps, recs, outs)

    def serve(self, reqs, arrivals_s: Sequence[float], keep_outputs: bool = False,
              staged=None, sleep_s: float = 50e-6) -> ServeResult:
        """Serve ``reqs`` arriving at ``arrivals_s`` (seconds after the start,
        non-decreasing).  Returns per-request latencies and tick statistics."""
        n = len(reqs)
        arrivals = np.asarray(arrivals_s, np.float64)
        if arrivals.shape != (n,) or (n and np.any(np.diff(arrivals) < 0)):
            raise ValueError("arrivals must be one non-decreasing time per request")
        sizes = [footprint_bytes(r) for r in reqs]
        work = [pair_count(r) for r in reqs]
        if staged is None:
            staged = [self.stage(r) for r in reqs]
        adm = Admission(self.budget, self.max_batch)
        stream = torch.cuda.current_stream(self.device)
        queue = collections.deque()
        inflight: collections.deque = collections.deque()
        done_ms = np.full(n, np.nan)
        tick_of = {}
        tick_events = []
        outputs = [None] * n if keep_outputs else None
        batch_sizes, rejected = [], []
        start = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(self.device)
        start.record(stream)
        t0 = time.perf_counter()
        nxt, finished = 0, 0

        def retire(tk):
            nonlocal finished
            adm.release(tk.bytes)
            finished += len(tk.ids)
            tk.held = None

        while finished + len(rejected) < n:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[nxt] <= now:
                queue.append(nxt)
                nxt += 1
            while inflight and inflight[0].event.query():
                retire(inflight.popleft())
            launched = False
            if queue and len(inflight) < self.depth:
                ids, rej = adm.admit(queue, sizes, work, self.max_tick_pairs)
                rejected.extend(rej)
                if ids:
                    outs, held = self._launch(reqs, staged, ids, stream)
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(stream)
                    tk = _Tick(ids, ev, held, sum(sizes[i] for i in ids))
                    inflight.append(tk)
                    tick_events.append(ev)
                    for i, o in zip(ids, outs):
                        tick_of[i] = len(tick_events) - 1
                        if keep_outputs:
                            outputs[i] = o
                    batch_sizes.append(len(ids))
                    launched = True
            if not launched:
                if inflight and (len(inflight) >= self.depth or not queue) and \
                        (nxt >= n or arrivals[nxt] > time.perf_counter() - t0 + 1e-3):
                    inflight[0].event.synchronize()
                elif sleep_s > 0:
                    time.sleep(sleep_s)
        while inflight:
            inflight[0].event.synchronize()
            retire(inflight.popleft())
        torch.cuda.synchronize(self.device)
        wall_ms = (time.perf_counter() - t0) * 1e3
        tick_ms = [start.elapsed_time(e) for e in tick_events]
        for i, k in tick_of.items():
            done_ms[i] = tick_ms[k]
        lat = done_ms - arrivals * 1e3
        makespan = float(np.nanmax(done_ms)) if np.isfinite(done_ms).any() else wall_ms
        return ServeResult(latency_ms=lat, done_ms=done_ms, makespan_ms=makespan, ticks=len(tick_events),
                           batch_sizes=batch_sizes, peak_bytes=adm.peak, rejected=rejected, outputs=outputs)


def poisson_arrivals(n: int, rate_per_s: float, seed: int = 0) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate."""
    if rate_per_s <= 0:
        raise ValueError("rate must be positive")
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, n))
