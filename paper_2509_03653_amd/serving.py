"""Serving loop: continuous batching of arriving packet windows.

Requests (one window of (src, dst) packets each, in host memory) arrive over
time.  The server

  * admits a request when its packets fit the device arena, a fixed ring of
    packet slots handed out in admission order (so the windows of a batch lie
    next to each other and form the offsets of one batched call), and
    uploads it on a copy stream;
  * launches, whenever fewer than `inflight` batches are on the device, one
    batched call over every admitted request not yet launched, on one of
    several compute streams, each ordered after its requests' uploads;
  * copies each batch's statistics back asynchronously and completes its
    requests when that copy has landed, then frees their arena slots (oldest
    first, so the ring stays contiguous).

Requests arriving while batches run are admitted as arena space frees up and
join the next batch: their uploads overlap the kernels in flight.  Latency is
measured from a request's arrival to its statistics being on the host, so it
includes admission wait, upload, queueing, compute and download.

The scheduling logic talks to an executor (`GpuExecutor` on the device; tests
substitute a host fake), so it can be exercised without a GPU.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


# ---- arena -------------------------------------------------------------------

class RingArena:
    """Packet slots [0, capacity) allocated contiguously in FIFO order.

    `alloc(n)` (n >= 1) returns the start of n consecutive free slots or None.
    When the slots left before the end are too few, the allocation starts
    again at 0 and the skipped tail stays reserved until it is freed.
    Allocations are marked done in any order; `release()` frees them from the
    oldest on while they are done, so the live slots always form one
    circular interval [tail, head).
    """

    def __init__(self, capacity: int):
        if capacity <= 0:
            raise ValueError("capacity must be positive")
        self.capacity = int(capacity)
        self.head = 0
        self.live = collections.deque()   # [start, n, reserved_from, done]

    def alloc(self, n: int):
        n = int(n)
        if n <= 0:
            raise ValueError("allocations take at least one slot")
        if n > self.capacity:
            raise ValueError(f"window of {n} packets exceeds the arena ({self.capacity})")
        cap, head = self.capacity, self.head
        start = reserved = 0           # reserved: where this allocation's slots begin
        if self.live:
            tail = self.live[0][2]
            if head > tail:            # free: [head, cap) and [0, tail)
                if cap - head >= n:
                    start = reserved = head
                elif tail >= n:        # wrap: the tail [head, cap) is skipped
                    start, reserved = 0, head
                else:
                    return None
            elif head < tail:          # free: [head, tail)
                if tail - head < n:
                    return None
                start = reserved = head
            else:                      # head == tail with live slots: full
                return None
        self.head = start + n
        self.live.append([start, n, reserved, False])
        return start

    def mark_done(self, start: int, n: int) -> None:
        for e in self.live:
            if e[0] == start and e[1] == n and not e[3]:
                e[3] = True
                return
        raise KeyError((start, n))

    def release(self) -> int:
        """Free done allocations from the oldest on; returns how many."""
        k = 0
        while self.live and self.live[0][3]:
            self.live.popleft()
            k += 1
        if not self.live:
            self.head = 0
        return k

    def in_use(self) -> int:
        """Slots reserved by live allocations (skipped tails included)."""
        if not self.live:
            return 0
        tail = self.live[0][2]
        return (self.head - tail) % self.capacity or self.capacity


# ---- requests ----------------------------------------------------------------

@dataclass
class Request:
    rid: int
    src: np.ndarray              # host packets (pinned torch tensors also work)
    dst: np.ndarray
    arrival: float = 0.0         # seconds on the server clock
    start: int = -1              # arena slot of the first packet
    admitted: float = -1.0
    completed: float = -1.0
    stats: np.ndarray = None     # (9,) uint64 once complete
    batch: int = -1

    @property
    def n(self) -> int:
        return int(len(self.src))

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


@dataclass
class Batch:
    bid: int
    reqs: list
    handle: object = None
    launched: float = 0.0


@dataclass
class ServeResult:
    requests: list
    batches: int
    wall: float
    first_arrival: float
    last_completion: float
    warmup: int = 0
    extra: dict = field(default_factory=dict)

    def measured(self):
        return sorted(self.requests, key=lambda r: r.rid)[self.warmup:]

    def summary(self) -> dict:
        m = self.measured()
        if not m:
            return {"windows": 0}
        lat = np.array([r.latency for r in m]) * 1e3
        t0 = min(r.arrival for r in m)
        t1 = max(r.completed for r in m)
        span = max(t1 - t0, 1e-9)
        pk = sum(r.n for r in m)
        return {"windows": len(m), "packets": int(pk), "seconds": span,
                "windows_per_s": len(m) / span, "packets_per_s": pk / span,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "batches": self.batches,
                "mean_batch_windows": len(self.requests) / max(self.batches, 1)}


# ---- scheduler -----------------------------------------------------------------

class Server:
    """Continuous-batching scheduler over an executor.

    executor API:
      upload(req)                        enqueue the copy of req's packets to
                                         arena slots [req.start, req.start+n)
      launch(reqs) -> handle             one batched call over the requests'
                                         (adjacent) slots, after their uploads
      poll(handle) -> bool               True once the statistics are on the host
      results(handle) -> (W, 9) uint64
    """

    def __init__(self, executor, arena_packets: int, inflight: int = 2,
                 max_batch_windows: int = 1024, max_batch_packets: int | None = None,
                 clock=time.perf_counter):
        streams = getattr(executor, "streams", None)
        if streams is not None and inflight > len(streams):
            raise ValueError("inflight batches exceed the executor's compute streams")
        self.ex = executor
        self.arena = RingArena(arena_packets)
        self.inflight = int(inflight)
        self.max_batch_windows = int(max_batch_windows)
        self.max_batch_packets = int(max_batch_packets or arena_packets)
        self.clock = clock
        self.pending = collections.deque()    # arrived, waiting for arena space
        self.staged = collections.deque()     # admitted + uploading, not launched
        self.running = collections.deque()    # launched batches, oldest first
        self.done = []
        self.nbatches = 0

    # -- steps --
    def _admit(self, now):
        while self.pending:
            r = self.pending[0]
            if r.n == 0:                 # empty windows take no slots
                self.pending.popleft()
                r.start, r.admitted = -1, now
                self.staged.append(r)
                continue
            start = self.arena.alloc(r.n)
            if start is None:
                return
            self.pending.popleft()
            r.start = start
            r.admitted = now
            self.ex.upload(r)
            self.staged.append(r)

    def _launch(self, now):
        while self.staged and len(self.running) < self.inflight:
            reqs = [self.staged.popleft()]
            pk = reqs[0].n
            end = reqs[0].start + reqs[0].n if reqs[0].n else None
            while self.staged and len(reqs) < self.max_batch_windows:
                r = self.staged[0]
                if r.n and ((end is not None and r.start != end) or pk + r.n > self.max_batch_packets):
                    break                # not adjacent in the arena, or batch full
                self.staged.popleft()
                reqs.append(r)
                if r.n:
                    pk += r.n
                    end = r.start + r.n
            b = Batch(self.nbatches, reqs, launched=now)
            for r in reqs:
                r.batch = b.bid
            self.nbatches += 1
            b.handle = self.ex.launch(reqs)
            self.running.append(b)

    def _complete(self, now) -> int:
        k = 0
        for b in list(self.running):
            if self.ex.poll(b.handle):
                out = self.ex.results(b.handle)
                for i, r in enumerate(b.reqs):
                    r.stats = np.asarray(out[i], dtype=np.uint64).copy()
                    r.completed = now
                    if r.n:
                        self.arena.mark_done(r.start, r.n)
                    self.done.append(r)
                self.running.remove(b)
                k += 1
        if k:
            self.arena.release()
        return k

    def step(self, arrivals=()):
        now = self.clock()
        for r in arrivals:
            self.pending.append(r)
        self._complete(now)
        self._admit(now)
        self._launch(now)

    def busy(self) -> bool:
        return bool(self.pending or self.staged or self.running)

    def run(self, requests, arrival_times=None, warmup: int = 0, timeout_s: float = 600.0):
        """Serve `requests`.  `arrival_times` (seconds after start, sorted) makes
        an open-loop run; None submits everything at once (closed loop, the
        saturation rate)."""
        reqs = list(requests)
        times = np.zeros(len(reqs)) if arrival_times is None else np.asarray(arrival_times, float)
        if len(times) != len(reqs):
            raise ValueError("one arrival time per request")
        order = np.argsort(times, kind="stable")
        t0 = self.clock()
        i = 0
        deadline = t0 + timeout_s
        while i < len(reqs) or self.busy():
            now = self.clock()
            if now > deadline:
                raise TimeoutError(f"serving did not finish within {timeout_s} s")
            arrived = []
            while i < len(reqs) and t0 + times[order[i]] <= now:
                r = reqs[order[i]]
                r.arrival = t0 + times[order[i]]
                arrived.append(r)
                i += 1
            self.step(arrived)
        t1 = self.clock()
        done = sorted(self.done, key=lambda r: r.rid)
        self.done = []
        return ServeResult(done, self.nbatches, t1 - t0, t0, max((r.completed for r in done), default=t0),
                           warmup=warmup)


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of `rate` per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


# ---- device executor -----------------------------------------------------------

class GpuExecutor:
    """Executor on one GPU: a device arena of `capacity` packet slots for src
    and dst, two copy streams (src and dst), `streams` compute streams (each with its library
    workspace reserved for the largest batch, so nothing is allocated while
    serving), and pinned result buffers."""

    def __init__(self, capacity: int, max_batch_windows: int, streams: int = 2, device=None):
        import torch

        import paper_2509_03653_amd as nsgc
        self.torch, self.nsgc = torch, nsgc
        self.dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.capacity = int(capacity)
        self.src = torch.empty(self.capacity, dtype=torch.int32, device=self.dev)
        self.dst = torch.empty(self.capacity, dtype=torch.int32, device=self.dev)
        # src and dst go up on two copy streams so that two DMA engines share
        # each window's upload
        self.copy_streams = [torch.cuda.Stream(self.dev), torch.cuda.Stream(self.dev)]
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(max(1, streams))]
        self.max_w = int(max_batch_windows)
        for s in self.streams:
            nsgc.reserve(self.capacity, self.max_w, stream=s)
        self.outs = [torch.empty((self.max_w, 9), dtype=torch.int64, device=self.dev)
                     for _ in self.streams]
        self.host = [torch.empty((self.max_w, 9), dtype=torch.int64, pin_memory=True)
                     for _ in self.streams]
        # a stream's buffers belong to its last batch until the scheduler has
        # taken that batch's results (the event alone is not enough: a batch
        # may finish between the scheduler's poll and its next launch)
        self.owner = [None] * len(self.streams)
        self.last_upload = [None, None]

    def upload(self, r):
        torch = self.torch
        n = r.n
        if n == 0:
            return
        src = r.src if isinstance(r.src, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(r.src).view(np.int32))
        dst = r.dst if isinstance(r.dst, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(r.dst).view(np.int32))
        for i, (buf, host) in enumerate(((self.src, src), (self.dst, dst))):
            cs = self.copy_streams[i]
            with torch.cuda.stream(cs):
                buf[r.start:r.start + n].copy_(host.view(torch.int32), non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(cs)
            self.last_upload[i] = ev

    def launch(self, reqs):
        torch = self.torch
        k = next((i for i, o in enumerate(self.owner) if o is None), None)
        if k is None:
            raise RuntimeError("more batches in flight than compute streams")
        s = self.streams[k]
        for ev in self.last_upload:         # uploads are in order on each copy stream
            if ev is not None:
                s.wait_event(ev)
        w = len(reqs)
        if w > self.max_w:
            raise ValueError("batch larger than the executor was sized for")
        first = next((r.start for r in reqs if r.n), 0)
        off = np.empty(w + 1, np.int64)
        off[0] = first
        off[1:] = first + np.cumsum([r.n for r in reqs])
        out = self.outs[k][:w]
        self.nsgc.window_stats(self.src, self.dst, off, out=out, stream=s)
        host = self.host[k][:w]
        with torch.cuda.stream(s):
            host.copy_(out, non_blocking=True)
        ev = torch.cuda.Event()
        ev.record(s)
        handle = (ev, host, k)
        self.owner[k] = handle
        return handle

    def poll(self, handle) -> bool:
        return handle[0].query()

    def results(self, handle):
        ev, host, k = handle
        ev.synchronize()
        out = host.numpy().view(np.uint64).copy()
        if self.owner[k] is handle:
            self.owner[k] = None            # the stream and its buffers are free again
        return out
