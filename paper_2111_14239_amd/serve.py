"""Continuous-batching server for the codec (host-side scheduling only).

Every step of the codec runs in the HIP library; this module decides what
runs when.  Requests are single device-resident images (a window of a
pre-staged device buffer) with their own (rho, alpha, r).  The server

* takes requests in order of their (scheduled) arrival time: open loop, so a
  server that falls behind accumulates latency instead of slowing arrivals;
* admits them first-in first-out as device memory for their reconstruction
  frees up in a fixed-size arena (first-fit, 256-byte aligned): a request
  larger than the whole arena is rejected;
* keeps S stream slots, each with its own reusable plan and results array; a
  free slot launches one batch of every admitted request at once (one
  persistent launch, plan updated asynchronously on the slot's stream), so
  work admitted while other batches run overlaps them on the device;
* polls the slots' completion events, hands each finished request's result
  (and its reconstruction, through a callback) back and frees its memory.

Latency of a request is completion time minus scheduled arrival time.
"""
from __future__ import annotations

import bisect
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import rklt


class Arena:
    """First-fit allocator of byte ranges in one device buffer."""

    def __init__(self, nbytes: int, align: int = 256):
        self.nbytes = int(nbytes)
        self.align = align
        self._free = [(0, self.nbytes)]  # sorted (offset, size)
        self._used: dict[int, int] = {}

    def alloc(self, n: int):
        n = (int(n) + self.align - 1) // self.align * self.align
        for k, (off, size) in enumerate(self._free):
            if size >= n:
                if size == n:
                    self._free.pop(k)
                else:
                    self._free[k] = (off + n, size - n)
                self._used[off] = n
                return off
        return None

    def free(self, off: int):
        n = self._used.pop(off)
        k = bisect.bisect_left(self._free, (off, 0))
        self._free.insert(k, (off, n))
        # merge with the neighbours
        if k + 1 < len(self._free) and off + n == self._free[k + 1][0]:
            self._free[k] = (off, n + self._free[k + 1][1])
            self._free.pop(k + 1)
        if k > 0 and self._free[k - 1][0] + self._free[k - 1][1] == self._free[k][0]:
            self._free[k - 1] = (self._free[k - 1][0], self._free[k - 1][1] + self._free[k][1])
            self._free.pop(k)

    @property
    def in_use(self) -> int:
        return sum(self._used.values())


@dataclass
class Request:
    arrival: float            # scheduled arrival, seconds from the start
    src: torch.Tensor         # 2D uint8 device view (may have a pitch)
    rho: float
    alpha: float
    r: int
    N: int = 8
    level_shift: int = 128
    tid: int = -1             # transform id; resolved before serving when -1
    # filled by the server
    admitted: float = float("nan")
    launched: float = float("nan")
    done: float = float("nan")
    result: dict = field(default_factory=dict)
    rejected: bool = False
    _off: int = -1
    _pitch: int = 0

    @property
    def pixels(self) -> int:
        return int(self.src.shape[0] * self.src.shape[1])


class _Slot:
    def __init__(self, max_batch: int, device):
        self.stream = torch.cuda.Stream(device=device)
        self.event = torch.cuda.Event()
        self.plan = None
        self.res = rklt.new_results(max_batch, device)
        self.res_host = torch.empty(max_batch * rklt.RESULT_BYTES, dtype=torch.uint8, pin_memory=True)
        self.batch: list[Request] | None = None


class Server:
    """Continuous batching over `streams` slots and an arena of `hbm_bytes`."""

    def __init__(self, ctx: rklt.Context, hbm_bytes: int, streams: int = 2, max_batch: int = 256,
                 device: int = 0, tuning=None):
        self.ctx = ctx
        self.device = torch.device("cuda", device)
        self.buf = torch.empty(int(hbm_bytes), dtype=torch.uint8, device=self.device)
        self.arena = Arena(hbm_bytes)
        self.max_batch = max_batch
        self.tuning = tuning
        self.slots = [_Slot(max_batch, self.device) for _ in range(streams)]
        self.batches = 0

    def _dst(self, req: Request) -> torch.Tensor:
        H, W = req.src.shape
        return self.buf[req._off:req._off + H * req._pitch].view(H, req._pitch)[:, :W]

    def _launch(self, slot: _Slot, batch: list[Request], now: float):
        descs = []
        for req in batch:
            descs.append(rklt.image_desc(req.src, req.tid, req.r, dst=self._dst(req), level_shift=req.level_shift))
        n = len(batch)
        with torch.cuda.stream(slot.stream):
            if slot.plan is None:
                slot.plan = self.ctx.plan(descs, self.tuning)
            else:
                slot.plan.update(descs, slot.stream)
            slot.plan.run(int(slot.res.data_ptr()), slot.stream)
            slot.res_host[:n * rklt.RESULT_BYTES].copy_(slot.res[:n * rklt.RESULT_BYTES], non_blocking=True)
            slot.event.record(slot.stream)
        for req in batch:
            req.launched = now
        slot.batch = batch
        self.batches += 1

    def serve(self, requests: list[Request], on_done=None, clock=time.perf_counter) -> dict:
        """Serve `requests` (sorted by arrival).  `on_done(request, dst)` is
        called with each finished request and a device view of its
        reconstruction, before that memory is reused.

        The transform of each distinct (N, rho, alpha) is designed on the host
        and uploaded before the clock starts (it is per-parameter set-up, not
        per-image work); requests whose design fails are rejected up front."""
        reqs = sorted(requests, key=lambda q: q.arrival)
        for req in reqs:
            W = int(req.src.shape[1])
            req._pitch = (W + rklt.ROW_ALIGN - 1) // rklt.ROW_ALIGN * rklt.ROW_ALIGN  # rows on 128-byte boundaries
            if req.tid < 0:
                try:
                    req.tid = self.ctx.transform_id(req.N, req.rho, req.alpha)
                except rklt.RkltError:
                    req.rejected = True
        pending: deque[Request] = deque()
        admitted: list[Request] = []
        i = 0
        finished = sum(1 for q in reqs if q.rejected)
        batches0 = self.batches
        t0 = clock()
        while finished < len(reqs):
            now = clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                if reqs[i].rejected:
                    reqs[i].done = now
                else:
                    pending.append(reqs[i])
                i += 1
            # admission, first in first out, by free arena memory
            while pending:
                req = pending[0]
                need = int(req.src.shape[0]) * req._pitch
                if need > self.arena.nbytes:
                    req.rejected = True
                    req.done = now
                    pending.popleft()
                    finished += 1
                    continue
                off = self.arena.alloc(need)
                if off is None:
                    break
                req._off = off
                req.admitted = now
                admitted.append(pending.popleft())
            # completions
            for slot in self.slots:
                if slot.batch is not None and slot.event.query():
                    t = clock() - t0
                    res = rklt.read_results(slot.res_host[:len(slot.batch) * rklt.RESULT_BYTES])
                    for req, r in zip(slot.batch, res):
                        req.done = t
                        req.result = r
                        if on_done is not None:
                            on_done(req, self._dst(req))
                        self.arena.free(req._off)
                        finished += 1
                    slot.batch = None
            # launches: a free slot takes every admitted request (up to max_batch)
            for slot in self.slots:
                if slot.batch is None and admitted:
                    batch, admitted = admitted[:self.max_batch], admitted[self.max_batch:]
                    self._launch(slot, batch, clock() - t0)
            if not admitted and not pending and all(s.batch is None for s in self.slots) and i < len(reqs):
                # idle until the next arrival
                wait = reqs[i].arrival - (clock() - t0)
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
        wall = clock() - t0
        return summarize(reqs, wall, self.batches - batches0)


def summarize(reqs: list[Request], wall: float, batches: int) -> dict:
    served = [q for q in reqs if not q.rejected]
    lat = np.array([q.done - q.arrival for q in served]) * 1e3
    px = sum(q.pixels for q in served)
    span = max(q.done for q in served) - min(q.arrival for q in served) if served else 0.0
    return {
        "requests": len(reqs), "served": len(served), "rejected": len(reqs) - len(served),
        "batches": batches, "wall_s": wall,
        "throughput_mpix_s": px / span / 1e6 if span > 0 else 0.0,
        "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
        "mean_batch": len(served) / max(batches, 1),
    }


def pool_requests(items, pool: list[torch.Tensor], pool_rhos: list[float]) -> list[Request]:
    """Requests from (arrival, ImageSpec) pairs: each one codes the top-left
    H x W window of the pre-staged device image whose correlation is nearest
    to the request's rho (the window is clipped to that image's size)."""
    out = []
    for t, spec in items:
        k = min(range(len(pool)), key=lambda j: abs(pool_rhos[j] - spec.rho))
        src = pool[k]
        H = min(spec.H, int(src.shape[0]))
        W = min(spec.W, int(src.shape[1]))
        out.append(Request(float(t), src[:H, :W], spec.rho, spec.alpha, spec.r, N=spec.N,
                           level_shift=spec.ell))
    return out
