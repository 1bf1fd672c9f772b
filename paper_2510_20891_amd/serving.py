"""Serving form: a request loop over device-resident spectrograms.

Scoring requests (a batch of coefficient vectors against one of several
resident data streams, returning its top-k) arrive from many search chains
at unpredictable times (Sec. II D: walkers propose candidates continuously).
The loop does continuous batching:

* admission -- a request is admitted once its device footprint (coefficients,
  statistic and top-k outputs) fits in what the HBM budget has left; larger
  ones wait in arrival order (no overtaking, so nothing starves);
* batching -- whenever one of ``slots`` in-flight slots is free, every admitted
  request that fits the slot (up to ``max_batch_templates``) is packed into
  one batched launch (one persistent kernel over all of them, each against
  its own spectrogram, each with its own top-k);
* overlap -- each slot has its own HIP stream, pinned staging buffer and
  device buffers, so a batch uploads, runs and returns its top-k while the
  batches of other slots are on the device;
* completion -- slots are polled with events; a request's latency is its
  completion (seen by the host) minus its arrival, on the host monotonic clock.

Each request's result is bit for bit the one a standalone score_tracks call
gives (the batched kernel sums every template in the same order).

The GPU side is an executor (``GpuExecutor``); the loop itself only needs
``launch(slot, requests)`` and ``poll(slot)``, so its admission and batching
logic can be tested on the CPU with a fake executor.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    stream: int                 # index of the resident spectrogram
    coeffs: np.ndarray          # (n, K) float32, host
    top_k: int
    t_arrival: float            # host monotonic seconds
    t_admit: float = math.nan
    t_done: float = math.nan
    topk_val: np.ndarray | None = None
    topk_idx: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.coeffs.shape[0])

    def device_bytes(self, K: int) -> int:
        n4 = (self.n + 3) // 4 * 4            # 16-byte aligned sub-buffers
        return n4 * (4 * K + 4) + self.top_k * 12

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class GpuExecutor:
    """Runs a batch of requests as one batched launch on a slot's stream."""

    def __init__(self, specs, f0s, Us, K: int, slots: int, max_batch_templates: int, max_requests: int,
                 top_k: int, precision: str = "plain"):
        import torch
        from . import Workspace
        self.specs, self.f0s, self.Us, self.K = specs, f0s, Us, int(K)
        self.precision, self.top_k = precision, int(top_k)
        dev = specs[0].data.device
        cap = int(max_batch_templates) + 4 * int(max_requests)
        self.streams = [torch.cuda.Stream() for _ in range(slots)]           # default priority
        self.h_coeffs = [torch.empty((cap, self.K), dtype=torch.float32, pin_memory=True) for _ in range(slots)]
        self.d_coeffs = [torch.empty((cap, self.K), dtype=torch.float32, device=dev) for _ in range(slots)]
        self.d_stat = [torch.empty(cap, dtype=torch.float32, device=dev) for _ in range(slots)]
        self.d_val = [torch.empty((max_requests, self.top_k), dtype=torch.float32, device=dev) for _ in range(slots)]
        self.d_idx = [torch.empty((max_requests, self.top_k), dtype=torch.int64, device=dev) for _ in range(slots)]
        self.h_val = [torch.empty((max_requests, self.top_k), dtype=torch.float32, pin_memory=True)
                      for _ in range(slots)]
        self.h_idx = [torch.empty((max_requests, self.top_k), dtype=torch.int64, pin_memory=True)
                      for _ in range(slots)]
        self.ws = [Workspace() for _ in range(slots)]
        self.events = [None] * slots
        self.batches = [None] * slots
        self.plans = [None] * slots
        # the per-slot problem tables, filled per batch with raw pointers into
        # the slot's buffers (same sub-buffers and 16-byte alignment as slices)
        from . import _Problem
        self.tables = [(_Problem * int(max_requests))() for _ in range(slots)]
        self.powers = [s_._struct() for s_ in specs]
        self.f0_ptr = [int(t.data_ptr()) for t in f0s]
        self.U_ptr = [int(t.data_ptr()) for t in Us]
        self.device = dev

    def launch(self, slot: int, reqs: list) -> None:
        import torch
        from . import RawBatchPlan
        st = self.streams[slot]
        K = self.K
        hc = self.h_coeffs[slot].numpy()
        tab = self.tables[slot]
        c0 = int(self.d_coeffs[slot].data_ptr())
        s0 = int(self.d_stat[slot].data_ptr())
        v0 = int(self.d_val[slot].data_ptr())
        i0 = int(self.d_idx[slot].data_ptr())
        off = 0
        for i, r in enumerate(reqs):
            n = r.n
            hc[off:off + n] = r.coeffs
            a = tab[i]
            a.power = self.powers[r.stream]
            a.f0 = self.f0_ptr[r.stream]
            a.U = self.U_ptr[r.stream] if K else None
            a.coeffs = c0 + 4 * K * off if K and n else None
            a.n_tmpl = n
            a.top_k = r.top_k
            a.k_min = 0
            a.k_max = -1
            a.stat = s0 + 4 * off if n else None
            a.topk_val = v0 + 4 * self.top_k * i if r.top_k else None
            a.topk_idx = i0 + 8 * self.top_k * i if r.top_k else None
            off += (n + 3) // 4 * 4
        with torch.cuda.stream(st):
            self.d_coeffs[slot][:off].copy_(self.h_coeffs[slot][:off], non_blocking=True)
            plan = RawBatchPlan(tab, len(reqs), K, precision=self.precision, workspace=self.ws[slot],
                                device=self.device, stream=st)
            plan.run(st)
            nr = len(reqs)
            self.h_val[slot][:nr].copy_(self.d_val[slot][:nr], non_blocking=True)
            self.h_idx[slot][:nr].copy_(self.d_idx[slot][:nr], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        self.events[slot], self.batches[slot], self.plans[slot] = ev, reqs, plan

    def poll(self, slot: int) -> bool:
        """True once the slot's batch is complete (results then filled in)."""
        ev = self.events[slot]
        if ev is None or not ev.query():
            return False
        for i, r in enumerate(self.batches[slot]):
            r.topk_val = self.h_val[slot][i, :r.top_k].numpy().copy()
            r.topk_idx = self.h_idx[slot][i, :r.top_k].numpy().copy()
        self.events[slot] = self.batches[slot] = self.plans[slot] = None
        return True


@dataclass
class ServeStats:
    n_requests: int
    wall_s: float
    evals: float
    latency_ms: dict = field(default_factory=dict)
    batches: int = 0
    mean_batch_requests: float = 0.0
    max_queue: int = 0


class Server:
    """Continuous-batching request loop (see the module docstring)."""

    def __init__(self, executor, K: int, hbm_budget: int, max_batch_templates: int, max_requests: int,
                 slots: int, seg_counts=None, clock=time.monotonic):
        self.ex, self.K = executor, int(K)
        self.hbm_budget, self.max_batch_templates = int(hbm_budget), int(max_batch_templates)
        self.max_requests, self.slots = int(max_requests), int(slots)
        self.clock = clock
        self.seg_counts = seg_counts
        self.waiting = collections.deque()     # arrived, not yet admitted (arrival order)
        self.admitted = collections.deque()    # admitted, not yet launched
        self.inflight = [None] * self.slots
        self.used_bytes = 0
        self.done = []
        self.batches = 0
        self.batch_sizes = []
        self.max_queue = 0

    def submit(self, req: Request) -> None:
        if req.n > self.max_batch_templates or req.device_bytes(self.K) > self.hbm_budget:
            raise ValueError(f"request {req.rid} of {req.n} templates can never fit")
        self.waiting.append(req)

    def _admit(self, now: float) -> None:
        while self.waiting:
            r = self.waiting[0]
            b = r.device_bytes(self.K)
            if self.used_bytes + b > self.hbm_budget:
                break                                   # keep arrival order: no overtaking
            self.waiting.popleft()
            self.used_bytes += b
            r.t_admit = now
            self.admitted.append(r)

    def _dispatch(self) -> None:
        for s in range(self.slots):
            if self.inflight[s] is not None or not self.admitted:
                continue
            batch, n = [], 0
            while self.admitted and len(batch) < self.max_requests:
                r = self.admitted[0]
                if batch and n + r.n > self.max_batch_templates:
                    break
                batch.append(self.admitted.popleft())
                n += (r.n + 3) // 4 * 4
            self.ex.launch(s, batch)
            self.inflight[s] = batch
            self.batches += 1
            self.batch_sizes.append(len(batch))

    def _complete(self, now: float) -> None:
        for s in range(self.slots):
            if self.inflight[s] is not None and self.ex.poll(s):
                for r in self.inflight[s]:
                    r.t_done = now
                    self.used_bytes -= r.device_bytes(self.K)
                    self.done.append(r)
                self.inflight[s] = None

    def step(self) -> None:
        now = self.clock()
        self._complete(now)
        self._admit(now)
        self._dispatch()
        self.max_queue = max(self.max_queue, len(self.waiting) + len(self.admitted))

    def busy(self) -> bool:
        return bool(self.waiting or self.admitted or any(b is not None for b in self.inflight))

    def run(self, requests: list, poll_s: float = 5e-5) -> list:
        """Release each request at its t_arrival (seconds from now) and serve until all are done."""
        t0 = self.clock()
        pending = sorted(requests, key=lambda r: r.t_arrival)
        for r in pending:
            r.t_arrival += t0
        i = 0
        while i < len(pending) or self.busy():
            now = self.clock()
            while i < len(pending) and pending[i].t_arrival <= now:
                self.submit(pending[i])
                i += 1
            self.step()
            if i < len(pending):
                wait = pending[i].t_arrival - self.clock()
                if wait > 0:
                    time.sleep(min(wait, poll_s))
            elif self.busy():
                time.sleep(poll_s)
        return self.done

    def stats(self, requests: list, warmup_s: float = 0.0) -> ServeStats:
        t_first = min(r.t_arrival for r in requests)
        measured = [r for r in requests if r.t_arrival - t_first >= warmup_s]
        lat = np.array([r.latency for r in measured]) * 1e3
        t_start = min(r.t_arrival for r in measured)
        t_end = max(r.t_done for r in measured)
        evals = float(sum(r.n * (self.seg_counts[r.stream] if self.seg_counts else 1) for r in measured))
        return ServeStats(
            n_requests=len(measured), wall_s=t_end - t_start, evals=evals,
            latency_ms={"p50": float(np.percentile(lat, 50)), "p90": float(np.percentile(lat, 90)),
                        "p99": float(np.percentile(lat, 99)), "max": float(lat.max()), "mean": float(lat.mean())},
            batches=self.batches, mean_batch_requests=float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            max_queue=self.max_queue)
