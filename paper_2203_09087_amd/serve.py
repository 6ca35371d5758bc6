"""Serving form: a continuous-batching loop over the ECC library.

Requests (one image each, already resident in device memory or given as a
device view to copy from) arrive over time.  The loop admits arrived requests in
arrival order as long as their device footprint (input copy + int64 output) fits
the memory budget and a lane is free, gathers the admitted requests of a lane
into one ``ecc_compute_batch`` call, and records one event per batch.  A request
may be written on any stream: ``submit`` notes the submitting (current) stream,
and the lane that takes the request waits on the device for the work that stream
holds at admission (no wait when that stream is already idle).  Several
lanes (each its own library context and HIP stream) let batches that were
admitted at different times run on the device at the same time, so requests that
arrive while others are on the GPU join the next batch instead of waiting for the
GPU to drain.  Outputs stay on the device; completion times are taken when the
loop sees a batch's event complete.

All computation is in the library; this module only schedules calls.
"""
from __future__ import annotations

import collections
import gc
import time
from dataclasses import dataclass, field

from . import ecc


@dataclass
class Request:
    """One ECC request.  ``source`` is a device tensor (any strides); ``value_range``
    as in ``ecc.make_image``.  Timing fields are host ``perf_counter`` seconds."""
    source: object
    nbins: int = 4096
    value_range: object = None
    t_arrival: float = 0.0
    t_admit: float = -1.0
    t_done: float = -1.0
    out: object = None
    image: object = None
    nbytes: int = 0
    lane: int = -1
    batch_size: int = 0
    device_ms: float = -1.0   # the batch's device time, from its timing events (-1: not timed)
    stream: object = None     # the stream the request was submitted on (set by submit)
    done: object = None       # event after the request's batch (wait on it to read out)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival

    @property
    def queue_wait(self) -> float:
        return self.t_admit - self.t_arrival


@dataclass
class _Lane:
    ctx: object
    stream: object
    inflight: collections.deque = field(default_factory=collections.deque)   # (start, end, [requests])


class Server:
    """Continuous-batching ECC server on one GPU.

    budget_bytes: device memory that admitted, unfinished requests may hold.
    max_batch:    most requests per library call.
    lanes:        independent (context, stream) pairs; at most ``max_inflight``
                  batches are outstanding per lane.
    device_timing: time every batch with a pair of events (each request's
                  ``device_ms``); off, the events only order work.

    Every lane's context reserves, at start, the scratch any admissible batch
    needs (up to ``max_batch`` images within the budget, ``max_nbins`` bins), so
    that no call grows it later: growing waits for the whole device.
    """

    def __init__(self, device=0, construction="vertex", budget_bytes=8 << 30, max_batch=64, lanes=2,
                 max_inflight=2, max_nbins=4096, device_timing=True):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.max_inflight = int(max_inflight)
        self.device_timing = bool(device_timing)
        self._ready = {}          # one reusable event per submitting stream
        self.lanes = [_Lane(ecc.Context(device, construction), torch.cuda.Stream(self.device))
                      for _ in range(lanes)]
        cus = torch.cuda.get_device_properties(self.device).multi_processor_count
        scratch, tables = ecc.batch_reserve_bytes(self.max_batch, self.budget, max_nbins, cus)
        for ln in self.lanes:
            ln.ctx.reserve(scratch, tables)
        self.pending = collections.deque()
        self.held = 0             # bytes held by admitted, unfinished requests
        self.peak_held = 0
        self.completed = []
        self.batches = 0

    def close(self):
        for ln in self.lanes:
            ln.ctx.close()

    # ------------------------------------------------------------ scheduling

    def submit(self, req: Request):
        """Queues a request that has arrived (its ``t_arrival`` is already set).  Its
        source may still be being written by work on the current stream."""
        src = req.source
        # what a batch takes (a bad request would fail the whole batch it joins)
        if not 2 <= src.dim() <= 4:
            raise ValueError(f"requests are 2D to 4D images (got {src.dim()} dimensions)")
        if not 1 <= req.nbins <= 65535:
            raise ValueError(f"nbins must be in [1, 65535] (got {req.nbins})")
        req.nbytes = src.numel() * src.element_size() + 8 * req.nbins
        if req.nbytes > self.budget:
            raise ValueError(f"request of {req.nbytes} bytes exceeds the budget of {self.budget}")
        req.stream = self.torch.cuda.current_stream(self.device)
        self.pending.append(req)

    def _reap(self, now: float) -> int:
        done = 0
        for ln in self.lanes:
            while ln.inflight and ln.inflight[0][1].query():
                start, end, reqs = ln.inflight.popleft()
                dms = start.elapsed_time(end) if self.device_timing else -1.0
                for r in reqs:
                    r.t_done = now
                    r.device_ms = dms
                    self.held -= r.nbytes
                    r.image = None          # the input copy can be released
                    r.stream = None
                    self.completed.append(r)
                done += len(reqs)
        return done

    def _admit(self, now: float) -> int:
        torch = self.torch
        started = 0
        for li, ln in enumerate(self.lanes):
            if not self.pending:
                break
            if len(ln.inflight) >= self.max_inflight:
                continue
            batch = []
            nbins = self.pending[0].nbins
            while (self.pending and len(batch) < self.max_batch and self.pending[0].nbins == nbins
                   and self.held + self.pending[0].nbytes <= self.budget):
                r = self.pending.popleft()
                self.held += r.nbytes
                batch.append(r)
            if not batch:
                break      # the head request waits for memory to free up
            self.peak_held = max(self.peak_held, self.held)
            start = torch.cuda.Event(enable_timing=self.device_timing)
            end = torch.cuda.Event(enable_timing=self.device_timing)
            # the sources were written on their submitting streams: the lane waits
            # for what each of them holds now, unless it is idle already
            for st in {r.stream.cuda_stream: r.stream for r in batch}.values():
                if not st.query():
                    ev = self._ready.get(st.cuda_stream)
                    if ev is None:
                        ev = self._ready[st.cuda_stream] = torch.cuda.Event()
                    ev.record(st)
                    ln.stream.wait_event(ev)
            with torch.cuda.stream(ln.stream):
                for r in batch:
                    r.t_admit = now
                    r.lane = li
                    r.batch_size = len(batch)
                    if r.source.is_contiguous():
                        r.image = r.source
                        # the lane reads memory the caller's stream allocated
                        r.image.record_stream(ln.stream)
                    else:
                        r.image = r.source.contiguous()
                    r.out = torch.empty(r.nbins, dtype=torch.int64, device=self.device)
                start.record(ln.stream)
            ln.ctx.compute_batch([r.image for r in batch], nbins,
                                 value_ranges=[r.value_range for r in batch],
                                 outs=[r.out for r in batch], stream=ln.stream)
            end.record(ln.stream)
            for r in batch:
                r.done = end
            ln.inflight.append((start, end, batch))
            self.batches += 1
            started += len(batch)
        return started

    def step(self) -> None:
        now = time.perf_counter()
        self._reap(now)
        self._admit(now)

    def busy(self) -> bool:
        return bool(self.pending) or any(ln.inflight for ln in self.lanes)

    def drain(self) -> None:
        while self.busy():
            self.step()

    # ------------------------------------------------------------- open loop

    def run_open_loop(self, arrivals, make_request):
        """Replays an arrival schedule (seconds from start, ascending): request i is
        submitted once its time has come; returns the completed requests in order.

        Python's cyclic garbage collector is paused while the loop runs (objects
        are still freed by reference counting): a full collection over the
        process's objects stalled the loop for about 56 ms."""
        was_enabled = gc.isenabled()
        gc.disable()
        try:
            t0 = time.perf_counter()
            i, n = 0, len(arrivals)
            while i < n or self.busy():
                now = time.perf_counter()
                while i < n and t0 + arrivals[i] <= now:
                    req = make_request(i)
                    req.t_arrival = t0 + arrivals[i]
                    self.submit(req)
                    i += 1
                self.step()
        finally:
            if was_enabled:
                gc.enable()
        done = sorted(self.completed, key=lambda r: r.t_arrival)
        self.completed = []
        return done


def latency_summary(reqs, wall_s: float) -> dict:
    """p50/p99 latency (ms), completed requests per second, and where the time of
    a request goes: queue wait (arrival to admission), the device time of its
    batch, and its batch size (p50/p99 each); for the slowest 1% of requests the
    same means."""
    import numpy as np
    lat = np.array([r.latency for r in reqs]) * 1e3
    wait = np.array([r.queue_wait for r in reqs]) * 1e3
    dev = np.array([r.device_ms for r in reqs])
    bs = np.array([r.batch_size for r in reqs])
    tail = lat >= np.percentile(lat, 99)

    def pq(x):
        return [round(float(np.percentile(x, 50)), 3), round(float(np.percentile(x, 99)), 3)]
    return {"requests": len(reqs), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3),
            "completed_per_s": round(len(reqs) / wall_s, 1),
            "queue_wait_ms_p50_p99": pq(wait), "batch_device_ms_p50_p99": pq(dev),
            "batch_size_p50_p99": pq(bs),
            "slowest_1pct": {"latency_ms": round(float(lat[tail].mean()), 3),
                             "queue_wait_ms": round(float(wait[tail].mean()), 3),
                             "batch_device_ms": round(float(dev[tail].mean()), 3),
                             "batch_size": round(float(bs[tail].mean()), 1)}}
