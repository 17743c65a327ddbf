"""Request loop for NTT jobs: admission by HBM footprint and continuous batching.

A request is one ciphertext-shaped job: ``polys`` polynomials of ``L`` limbs at ring
degree ``N`` that need the forward transform, a product with a key polynomial kept
resident on the device in the NTT domain, and the inverse transform (the NTT-based
negacyclic product of Section III-A, applied to every RNS limb).  The loop:

* admits arrived requests in FIFO order while their footprint (the bytes of their
  residues) fits in a fixed device arena; twiddle tables and keys are resident and not
  counted against it;
* launches all admitted requests that are not yet running as one batch (forward,
  key product and inverse per plan) on a free stream lane, so work that arrives while
  other batches run is picked up as soon as a lane frees, and batches on different
  lanes overlap on the device;
* frees a request's memory when its batch has completed, recording the device-side
  completion time.

The ``per_request`` policy is the plain path to compare against: every request is
enqueued as soon as it is admitted, on one stream, with its own launches.

All arithmetic runs in the library's kernels; this module only orders work.  The
executor is injectable so that the scheduling logic can be exercised without a GPU.
"""
from __future__ import annotations

import bisect
import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Optional

__all__ = ["Request", "FootprintPool", "ServeStats", "Server", "GpuExecutor", "percentile"]

ALIGN = 256


@dataclass
class Request:
    rid: int
    N: int
    L: int
    arrival: float                    # seconds after the start of the run
    polys: int = 2
    payload: object = None            # input residues [polys][L][N] (device tensor for the GPU executor)
    # filled in by the server
    status: str = "pending"           # pending | done | rejected | failed
    error: str = ""
    offset: int = -1
    admit_t: float = math.nan
    launch_t: float = math.nan
    done_t: float = math.nan
    batch_id: int = -1

    @property
    def words(self) -> int:
        return self.polys * self.L * self.N

    @property
    def latency(self) -> float:
        return self.done_t - self.arrival


class FootprintPool:
    """First-fit allocator over a byte range [0, capacity) with coalescing frees.

    Offsets and sizes are multiples of ``align``.  ``alloc`` returns None when no free
    block is large enough (the caller keeps the request waiting)."""

    def __init__(self, capacity: int, align: int = ALIGN):
        if capacity <= 0 or align <= 0 or align & (align - 1):
            raise ValueError("capacity must be positive and align a power of two")
        self.align = align
        self.capacity = capacity - capacity % align
        self._starts = [0]                # free blocks, sorted by start
        self._sizes = {0: self.capacity}
        self._live: dict[int, int] = {}
        self.used = 0
        self.peak = 0

    def size_of(self, nbytes: int) -> int:
        return (nbytes + self.align - 1) // self.align * self.align

    def alloc(self, nbytes: int) -> Optional[int]:
        need = self.size_of(max(1, nbytes))
        for i, s in enumerate(self._starts):
            size = self._sizes[s]
            if size < need:
                continue
            del self._sizes[s]
            if size == need:
                self._starts.pop(i)
            else:
                self._starts[i] = s + need
                self._sizes[s + need] = size - need
            self._live[s] = need
            self.used += need
            self.peak = max(self.peak, self.used)
            return s
        return None

    def free(self, offset: int) -> None:
        size = self._live.pop(offset)     # KeyError on a double free
        self.used -= size
        i = bisect.bisect_left(self._starts, offset)
        start, end = offset, offset + size
        if i < len(self._starts) and self._starts[i] == end:           # merge with the next block
            end += self._sizes.pop(self._starts.pop(i))
        if i > 0 and self._starts[i - 1] + self._sizes[self._starts[i - 1]] == start:  # and the previous
            start = self._starts[i - 1]
            self._sizes[start] = end - start
        else:
            self._starts.insert(i, start)
            self._sizes[start] = end - start

    def largest_free(self) -> int:
        return max(self._sizes.values(), default=0)

    def check(self) -> None:
        """Invariants: free blocks sorted, disjoint, non-adjacent; free + live = capacity."""
        prev_end = -1
        for s in self._starts:
            assert s > prev_end, "free blocks overlap or touch"
            prev_end = s + self._sizes[s]
        assert set(self._starts) == set(self._sizes)
        assert sum(self._sizes.values()) + sum(self._live.values()) == self.capacity
        assert self.used == sum(self._live.values())


def percentile(xs, p: float) -> float:
    """Nearest-rank percentile (p in [0, 100]); NaN for an empty list."""
    xs = sorted(xs)
    if not xs:
        return math.nan
    k = max(0, min(len(xs) - 1, math.ceil(p / 100.0 * len(xs)) - 1))
    return xs[k]


@dataclass
class ServeStats:
    policy: str
    completed: int
    rejected: int
    failed: int
    batches: int
    mean_batch: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    max_ms: float
    throughput_rps: float             # completed requests / (last completion - first arrival)
    span_s: float
    peak_bytes: int
    capacity_bytes: int
    extra: dict = field(default_factory=dict)

    def as_dict(self) -> dict:
        d = dict(self.__dict__)
        d.update(d.pop("extra"))
        return d


class Server:
    """Runs a list of requests through an executor (see ``GpuExecutor`` for the protocol).

    policy "continuous": at most ``executor.lanes`` batches in flight; every admitted
    request that is not running joins the next batch (up to ``max_batch`` requests).
    policy "per_request": each request is launched alone as soon as it is admitted, on
    lane 0, with no limit on the number in flight (the stream orders them)."""

    def __init__(self, executor, capacity_bytes: int, policy: str = "continuous", max_batch: int = 256,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
                 idle_sleep: float = 20e-6):
        if policy not in ("continuous", "per_request"):
            raise ValueError(f"unknown policy {policy!r}")
        self.ex = executor
        self.pool = FootprintPool(capacity_bytes)
        self.policy = policy
        self.max_batch = max(1, int(max_batch))
        self.clock = clock
        self.sleep = sleep
        self.idle_sleep = idle_sleep

    def run(self, requests, on_complete: Optional[Callable[[Request, object], None]] = None) -> ServeStats:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        pending = deque(reqs)
        waiting: deque[Request] = deque()       # arrived, not yet admitted
        ready: deque[Request] = deque()         # admitted, not yet launched
        inflight: list[tuple[object, int, list[Request]]] = []
        busy = [False] * self.ex.lanes
        n_batches = 0
        batch_sizes = []
        t0 = self.ex.start(self.clock)

        def finish(reqs_, status, err=""):
            for r in reqs_:
                r.status = status
                r.error = err
                if r.offset >= 0:
                    self.pool.free(r.offset)
                    r.offset = -1

        while pending or waiting or ready or inflight:
            progressed = False
            # completions
            still = []
            for tok, lane, batch in inflight:
                if self.ex.poll(tok):
                    t_done = self.ex.finish_time(tok)
                    for r in batch:
                        r.done_t = t_done
                        if on_complete is not None:
                            on_complete(r, self.ex.view(r))
                    finish(batch, "done")
                    if self.policy == "continuous":
                        busy[lane] = False
                    progressed = True
                else:
                    still.append((tok, lane, batch))
            inflight = still
            now = self.clock() - t0
            # arrivals
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                err = self.ex.validate(r)
                if not err and self.pool.size_of(self.ex.footprint(r)) > self.pool.capacity:
                    err = "footprint exceeds the whole arena"
                if err:
                    r.status, r.error = "rejected", err
                else:
                    waiting.append(r)
                progressed = True
            # admission: FIFO, so a large request is not overtaken indefinitely
            while waiting:
                r = waiting[0]
                off = self.pool.alloc(self.ex.footprint(r))
                if off is None:
                    break
                waiting.popleft()
                r.offset, r.admit_t = off, now
                ready.append(r)
                progressed = True
            # launches
            while ready:
                if self.policy == "continuous":
                    lane = next((i for i, b in enumerate(busy) if not b), -1)
                    if lane < 0:
                        break
                    batch = [ready.popleft() for _ in range(min(self.max_batch, len(ready)))]
                else:
                    lane, batch = 0, [ready.popleft()]
                for r in batch:
                    r.launch_t, r.batch_id = now, n_batches
                try:
                    tok = self.ex.launch(lane, batch)
                except Exception as e:            # the batch fails alone; the loop goes on
                    finish(batch, "failed", f"{type(e).__name__}: {e}")
                    progressed = True
                    continue
                n_batches += 1
                batch_sizes.append(len(batch))
                if self.policy == "continuous":
                    busy[lane] = True
                inflight.append((tok, lane, batch))
                progressed = True
            if not progressed:
                wait = self.idle_sleep
                if pending and not inflight and not ready:
                    wait = max(wait, min(pending[0].arrival - now, 1e-3))
                self.sleep(wait)

        done = [r for r in reqs if r.status == "done"]
        lat = [r.latency * 1e3 for r in done]
        span = (max(r.done_t for r in done) - min(r.arrival for r in done)) if done else 0.0
        return ServeStats(
            policy=self.policy, completed=len(done),
            rejected=sum(r.status == "rejected" for r in reqs), failed=sum(r.status == "failed" for r in reqs),
            batches=n_batches, mean_batch=(sum(batch_sizes) / len(batch_sizes)) if batch_sizes else 0.0,
            p50_ms=percentile(lat, 50), p99_ms=percentile(lat, 99),
            mean_ms=(sum(lat) / len(lat)) if lat else math.nan, max_ms=max(lat) if lat else math.nan,
            throughput_rps=(len(done) / span) if span > 0 else math.nan, span_s=span,
            peak_bytes=self.pool.peak, capacity_bytes=self.pool.capacity)


class GpuExecutor:
    """Runs request batches through the library's batch API on ``lanes`` streams.

    plans: {N: Plan} sharing one prime chain (a request of L limbs uses its first L
    primes); keys: {N: device tensor [L_max][N]} in the NTT domain, resident.  The arena
    is one device tensor of ``capacity_bytes`` that the server's pool hands out.
    ``mode`` is the NTT_BATCH_* mode of each launch (grouped for continuous batching,
    plain for the per-request path)."""

    def __init__(self, plans: dict, keys: dict, capacity_bytes: int, lanes: int = 2, mode: Optional[int] = None,
                 device: str = "cuda"):
        import torch
        from . import BATCH_GROUPED, OP_FORWARD, OP_INVERSE, OP_MULKEY
        self.torch = torch
        self.plans = dict(plans)
        self.keys = dict(keys)
        for n, p in self.plans.items():
            if p.N != n:
                raise ValueError(f"plan for N={n} has N={p.N}")
            k = self.keys.get(n)
            if k is None or k.numel() < p.L * n or not k.is_contiguous():
                raise ValueError(f"missing or short key for N={n}")
        self.lanes = int(lanes)
        self.mode = BATCH_GROUPED if mode is None else mode
        self.op = OP_FORWARD | OP_MULKEY | OP_INVERSE
        self.arena = torch.empty(capacity_bytes // 8, dtype=torch.int64, device=device)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(self.lanes)]
        self._free_batches: list = []
        self._t0_event = None
        self._t0 = 0.0

    # -- protocol used by Server
    def validate(self, r: Request) -> str:
        p = self.plans.get(r.N)
        if p is None:
            return f"no plan for N={r.N}"
        if not 1 <= r.L <= p.L:
            return f"L={r.L} outside [1, {p.L}]"
        if r.polys < 1:
            return "polys must be positive"
        if r.payload is not None and tuple(r.payload.shape) != (r.polys, r.L, r.N):
            return f"payload shape {tuple(r.payload.shape)} != {(r.polys, r.L, r.N)}"
        return ""

    def footprint(self, r: Request) -> int:
        return 8 * r.words

    def start(self, clock) -> float:
        torch = self.torch
        torch.cuda.synchronize()
        self._t0_event = torch.cuda.Event(enable_timing=True)
        self._t0_event.record(self.streams[0])
        self._t0_event.synchronize()
        self._t0 = clock()
        return self._t0

    def view(self, r: Request):
        w0 = r.offset // 8
        return self.arena[w0:w0 + r.words].view(r.polys, r.L, r.N)

    def launch(self, lane: int, batch: list):
        from . import ntt_batch_assign, ntt_batch_create, ntt_batch_run
        torch = self.torch
        st = self.streams[lane]
        jobs = []
        with torch.cuda.stream(st):
            for r in batch:
                v = self.view(r)
                if r.payload is not None:
                    v.copy_(r.payload, non_blocking=True)
                p = self.plans[r.N]
                jobs.append((p, v, r.polys, r.L if r.L < p.L else 0, self.op, self.keys[r.N]))
        if self._free_batches:
            b = self._free_batches.pop()
            ntt_batch_assign(b, jobs, st)
        else:                                   # create uploads its descriptors synchronously
            b = ntt_batch_create(jobs)
        ntt_batch_run(b, self.mode, st)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(st)
        return (ev, b)

    def poll(self, tok) -> bool:
        ev, b = tok
        if not ev.query():
            return False
        self._free_batches.append(b)
        return True

    def finish_time(self, tok) -> float:
        ev, _ = tok
        return self._t0_event.elapsed_time(ev) / 1e3

    def close(self) -> None:
        self.torch.cuda.synchronize()
        for b in self._free_batches:
            b.destroy()
        self._free_batches.clear()
