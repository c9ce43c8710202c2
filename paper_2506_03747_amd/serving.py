"""Continuous-batching serving loop for the transient NLOS forward operator.

Requests (a depth map with its albedo and mask, plus system parameters)
arrive over time.  Whenever a tick slot is free, the server admits waiting
requests in arrival order while their device footprint fits in an HBM
budget, uploads their maps and runs the whole path for all of them -- depth
maps to records to jittered histograms -- as one serving tick: one launch of
a HIP graph instantiated once per slot (a table copy and three kernels over
a device work list, see nlos_tick_graph_* in nlos.h).  This is the K-frame
loop of Algorithm 1 with many scenes per frame.  Records and histograms stay
on the device; a request's bytes return to the budget when its tick's
completion event has passed.

Each slot has its own stream (all at the default priority), table and
workspace, so a tick admitted while others run starts at once: its work
overlaps theirs on the device instead of waiting for a tick boundary.

``mode="plain"`` serves the same stream one request at a time through the
single-request call (nlos_simulate) on one stream: the baseline that batching
is measured against.  Every request computes exactly what it computes alone.

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

from . import NlosError, TickGraph, n_histograms, params_of, simulate, tick_supported
from ._native import NLOS_RECORD_FLOATS

RECORD_BYTES = 4 * NLOS_RECORD_FLOATS
# one-call workspace per pixel: the records' pair-loop constants (32 B), the
# summaries (32 B per 256 records) and the block counts (4 B per 256-pixel
# block), rounded up
SIM_WS_PER_PIXEL = 32.0 + 32.0 / 256.0 + 8.0 / 256.0


def _pixels(req) -> int:
    return int(req.patch_grid["nx"]) * int(req.patch_grid["ny"])


def footprint_bytes(req, with_workspace: bool = True) -> int:
    """Device bytes a request holds while in flight: its maps, its patch
    records, its output histograms and (``with_workspace``) the one-call
    workspace it needs when served alone."""
    npx = _pixels(req)
    maps = 4 * npx + (4 * npx if req.albedo is not None else 0) + (npx if req.mask is not None else 0)
    rec = RECORD_BYTES * npx + 4
    out = 4 * n_histograms(params_of(req)) * int(req.n_bins)
    ws = int(SIM_WS_PER_PIXEL * npx) + 4096 if with_workspace else 0
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
              max_work: float = float("inf"), pixels: Optional[Sequence[int]] = None,
              max_pixels: float = float("inf")):
        """Pop admitted request ids from the head of ``queue``; returns
        (admitted, rejected).  With ``work`` (``pixels``) given, a tick also
        stops once its work (pixels) would pass ``max_work`` (``max_pixels``);
        its first request is always taken unless it alone passes
        ``max_pixels``, which rejects it."""
        admitted, rejected = [], []
        w, px = 0.0, 0
        while queue and len(admitted) < self.max_batch:
            i = queue[0]
            b = int(sizes[i])
            p = int(pixels[i]) if pixels is not None else 0
            if b > self.budget or p > max_pixels:
                queue.popleft()
                rejected.append(i)
                continue
            if self.in_use + b > self.budget:
                break
            if admitted and ((work is not None and w + float(work[i]) > max_work) or px + p > max_pixels):
                break
            queue.popleft()
            self.in_use += b
            admitted.append(i)
            if work is not None:
                w += float(work[i])
            px += p
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
    peak_bytes: int               # admitted request bytes in flight, at most
    fixed_bytes: int              # the server's own device buffers (tick workspaces)
    launches: List[int]           # host launches (graph launches and kernel launches) per tick
    rejected: List[int]
    outputs: Optional[list]       # per request device outputs (keep_outputs=True)

    def percentile(self, q: float) -> float:
        v = self.latency_ms[np.isfinite(self.latency_ms)]
        return float(np.percentile(v, q)) if v.size else float("nan")


class _Tick:
    __slots__ = ("ids", "event", "held", "bytes", "slot")

    def __init__(self, ids, event, held, nbytes, slot):
        self.ids = ids
        self.event = event
        self.held = held
        self.bytes = nbytes
        self.slot = slot


# Launches of one request served alone through nlos_simulate: geometry count
# and scatter, the pair kernel (the scan kernel past 4096 blocks, the zero
# fill when patches are split are not counted).
PLAIN_LAUNCHES = 3


class Server:
    """One GPU, continuous batching under an HBM budget.

    budget_bytes    device bytes the server may hold: its tick workspaces and
                    the footprints of the requests in flight.
    max_batch       requests per tick.
    depth           ticks in flight (batched: tick slots, each with its own
                    stream, table, workspace and graph).
    max_tick_pairs  work per tick (pairs; the first request of a tick is
                    always taken): short ticks let requests complete soon
                    after their own work instead of at the end of a long tick.
    tick_pixels     depth-map pixels per tick (sizes each slot's workspace).
    Requests a tick cannot run (non-confocal, windowed plans) are served
    through nlos_simulate on the slot's stream.  mode="plain": one request
    per tick through nlos_simulate, on one stream."""

    def __init__(self, budget_bytes: int = 2 << 30, max_batch: int = 32, depth: int = 3,
                 mode: str = "batched", device="cuda", max_tick_pairs: float = 1e9,
                 tick_pixels: int = 1 << 21):
        if mode not in ("batched", "plain"):
            raise ValueError("mode is 'batched' or 'plain'")
        self.mode = mode
        self.device = torch.device(device)
        self.depth = max(1, int(depth))
        self.max_tick_pairs = float(max_tick_pairs)
        self.budget = int(budget_bytes)
        self.max_batch = 1 if mode == "plain" else int(max_batch)
        self.tick_pixels = int(tick_pixels)
        self.slots = []
        self.streams = []
        if mode == "batched":
            for _ in range(self.depth):
                self.slots.append(TickGraph(self.max_batch, self.tick_pixels, self.device))
                self.streams.append(torch.cuda.Stream(self.device))
        self.fixed_bytes = sum(s.bytes for s in self.slots)
        if self.fixed_bytes >= self.budget:
            raise ValueError("the budget does not cover the tick workspaces")

    @staticmethod
    def stage(req):
        """Host payload of a request in pinned memory (done as a request is
        received, before it is queued)."""
        pin = lambda a, dt: None if a is None else torch.from_numpy(np.ascontiguousarray(a, dt)).pin_memory()
        return (pin(req.depth, np.float32), pin(req.albedo, np.float32), pin(req.mask, np.uint8))

    def _upload(self, reqs, staged, ids):
        maps = []
        for i in ids:
            d, a, m = staged[i]
            maps.append(dict(params=params_of(reqs[i]), grid=reqs[i].patch_grid,
                             depth=d.to(self.device, non_blocking=True),
                             albedo=None if a is None else a.to(self.device, non_blocking=True),
                             mask=None if m is None else m.to(self.device, non_blocking=True)))
        return maps

    def _launch_batched(self, reqs, staged, ids, slot, stream, tickable):
        """Upload the maps and run the tick on the slot's stream; returns
        (outputs, held tensors, launches, completion event)."""
        with torch.cuda.stream(stream):
            maps = self._upload(reqs, staged, ids)
            in_tick = [k for k, i in enumerate(ids) if tickable[i]]
            outs = [None] * len(ids)
            launches = 0
            held = [maps]
            if in_tick:
                try:
                    res = slot.plan([maps[k] for k in in_tick])
                except NlosError:
                    in_tick = []   # served one by one below
                else:
                    slot.launch(stream)
                    launches += 1
                    held.append(res)
                    for k, (o, _, _) in zip(in_tick, res):
                        outs[k] = o
            for k, mp in enumerate(maps):
                if outs[k] is None:
                    o, p, n = simulate(mp["params"], mp["depth"], mp["grid"], mp["albedo"], mp["mask"],
                                       stream=stream)
                    outs[k] = o
                    held.append((o, p, n))
                    launches += PLAIN_LAUNCHES
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
        return outs, held, launches, ev

    def _launch_plain(self, reqs, staged, ids, stream):
        maps = self._upload(reqs, staged, ids)
        outs, held = [], [maps]
        for mp in maps:
            o, p, n = simulate(mp["params"], mp["depth"], mp["grid"], mp["albedo"], mp["mask"], stream=stream)
            outs.append(o)
            held.append((o, p, n))
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(stream)
        return outs, held, PLAIN_LAUNCHES * len(ids), ev

    def serve(self, reqs, arrivals_s: Sequence[float], keep_outputs: bool = False,
              staged=None, sleep_s: float = 50e-6) -> ServeResult:
        """Serve ``reqs`` arriving at ``arrivals_s`` (seconds after the start,
        non-decreasing).  Returns per-request latencies and tick statistics."""
        n = len(reqs)
        arrivals = np.asarray(arrivals_s, np.float64)
        if arrivals.shape != (n,) or (n and np.any(np.diff(arrivals) < 0)):
            raise ValueError("arrivals must be one non-decreasing time per request")
        batched = self.mode == "batched"
        # requests a tick runs (the rest go through the one-call path, with
        # its workspace in their footprint)
        tickable = [batched and _pixels(r) <= self.tick_pixels and tick_supported(params_of(r), r.patch_grid)
                    for r in reqs]
        sizes = [footprint_bytes(r, with_workspace=not t) for r, t in zip(reqs, tickable)]
        work = [pair_count(r) for r in reqs]
        pixels = [_pixels(r) if t else 0 for r, t in zip(reqs, tickable)] if batched else None
        if staged is None:
            staged = [self.stage(r) for r in reqs]
        adm = Admission(self.budget - self.fixed_bytes, self.max_batch)
        main = torch.cuda.current_stream(self.device)
        queue = collections.deque()
        inflight: List[_Tick] = []
        done_ms = np.full(n, np.nan)
        tick_of = {}
        tick_events = []
        outputs = [None] * n if keep_outputs else None
        batch_sizes, rejected, launches = [], [], []
        start = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(self.device)
        start.record(main)
        if batched:
            # every slot's stream starts after the start event
            for s in self.streams:
                s.wait_stream(main)
        t0 = time.perf_counter()
        nxt, finished = 0, 0

        def retire(tk):
            nonlocal finished
            adm.release(tk.bytes)
            finished += len(tk.ids)
            tk.held = None
            inflight.remove(tk)

        def free_slot():
            if not batched:
                return 0 if len(inflight) < self.depth else None
            used = {tk.slot for tk in inflight}
            for k in range(len(self.slots)):
                if k not in used:
                    return k
            return None

        while finished + len(rejected) < n:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[nxt] <= now:
                queue.append(nxt)
                nxt += 1
            for tk in [tk for tk in inflight if tk.event.query()]:
                retire(tk)
            launched = False
            k = free_slot() if queue else None
            if k is not None:
                ids, rej = adm.admit(queue, sizes, work, self.max_tick_pairs, pixels,
                                     self.tick_pixels if batched else float("inf"))
                rejected.extend(rej)
                if ids:
                    if batched:
                        outs, held, nl_, ev = self._launch_batched(reqs, staged, ids, self.slots[k],
                                                                   self.streams[k], tickable)
                    else:
                        outs, held, nl_, ev = self._launch_plain(reqs, staged, ids, main)
                    inflight.append(_Tick(ids, ev, held, sum(sizes[i] for i in ids), k))
                    tick_events.append(ev)
                    for i, o in zip(ids, outs):
                        tick_of[i] = len(tick_events) - 1
                        if keep_outputs:
                            outputs[i] = o
                    batch_sizes.append(len(ids))
                    launches.append(nl_)
                    launched = True
            if not launched:
                if inflight and (free_slot() is None or not queue) and \
                        (nxt >= n or arrivals[nxt] > time.perf_counter() - t0 + 1e-3):
                    oldest = min(inflight, key=lambda tk: tick_of[tk.ids[0]])
                    oldest.event.synchronize()
                elif sleep_s > 0:
                    time.sleep(sleep_s)
        while inflight:
            inflight[0].event.synchronize()
            retire(inflight[0])
        torch.cuda.synchronize(self.device)
        wall_ms = (time.perf_counter() - t0) * 1e3
        tick_ms = [start.elapsed_time(e) for e in tick_events]
        for i, kk in tick_of.items():
            done_ms[i] = tick_ms[kk]
        lat = done_ms - arrivals * 1e3
        makespan = float(np.nanmax(done_ms)) if np.isfinite(done_ms).any() else wall_ms
        return ServeResult(latency_ms=lat, done_ms=done_ms, makespan_ms=makespan, ticks=len(tick_events),
                           batch_sizes=batch_sizes, peak_bytes=adm.peak, fixed_bytes=self.fixed_bytes,
                           launches=launches, rejected=rejected, outputs=outputs)


def poisson_arrivals(n: int, rate_per_s: float, seed: int = 0) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate."""
    if rate_per_s <= 0:
        raise ValueError("rate must be positive")
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, n))
