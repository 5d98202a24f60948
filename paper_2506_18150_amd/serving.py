"""Continuous-batching request loop for encrypted lookups.

A request carries one selector ciphertext per touched table group (the
tables are split into fixed groups, one packed plan per group, so requests
of different table counts carry different amounts of work).  The server

* admits a request when its in-flight device bytes (selector and result
  ciphertexts) fit the HBM budget left after keys, plans and the per-stream
  workspaces (``helrm_footprint``); otherwise it waits, and it is rejected
  after ``admit_timeout`` seconds;
* keeps admitted work units (request, group, ciphertext) in per-group
  queues and, whenever one of its streams is free, launches a batch of up to
  ``max_batch`` units of the group whose oldest unit has waited longest --
  units of different requests share a batch, and batches on different
  streams overlap on the device; with ``mix_groups`` a batch takes the oldest
  units of any groups and one launch (helrm_lookup_batch) runs each through
  its own group's plan;
* completes a request when its last unit finishes and its results are on the
  host; latency = completion - arrival;
* cancels a request whose ``deadline`` (seconds after arrival) passes before
  it completes, or that the client withdraws (``cancel``): it leaves the
  admission queue, its queued units leave the group queues and its device
  bytes are released at once; units already running finish and their results
  are dropped.

The executor does the device work; ``GpuExecutor`` runs helrm_lookup_packed
on HIP streams, ``FakeExecutor`` (with ``FakeClock``) models durations so the
scheduler can be tested on a CPU.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Deque, Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float
    units: List[Tuple[int, Any]]            # (group, selector ciphertext payload)
    deadline: Optional[float] = None         # seconds after arrival; None = no deadline
    admitted_at: Optional[float] = None
    done_at: Optional[float] = None
    results: Dict[int, Any] = field(default_factory=dict)
    remaining: int = 0
    rejected: bool = False
    cancelled: Optional[str] = None          # "deadline" or "client" once cancelled
    bytes_in_flight: int = 0

    @property
    def closed(self) -> bool:
        return self.rejected or self.cancelled is not None

    @property
    def latency(self) -> Optional[float]:
        return None if self.done_at is None else self.done_at - self.arrival


@dataclass
class Unit:
    req: Request
    group: int
    payload: Any
    enq: float


class RealClock:
    def now(self) -> float:
        return time.perf_counter()

    def sleep_until(self, t: float) -> None:
        d = t - time.perf_counter()
        if d > 0:
            time.sleep(min(d, 0.002))


class FakeClock:
    """Time advances only when the loop waits for the next event."""

    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def sleep_until(self, t: float) -> None:
        if t > self.t:
            self.t = t


class Executor:
    n_streams: int

    def admit(self, req: Request) -> None:
        """Make an admitted request's selectors resident (device pool)."""

    def release(self, req: Request) -> None:
        """Free what admit() took for the request."""

    def unit_bytes(self, group: int) -> int: ...
    def static_bytes(self) -> int: ...
    def workspace_bytes(self, group: int, batch: int) -> int: ...
    def launch(self, stream: int, group: int, units: Sequence[Unit]) -> Any: ...
    def done(self, handle) -> bool: ...
    def next_done_time(self) -> Optional[float]: ...
    def results(self, handle) -> List[Any]: ...


class FakeExecutor(Executor):
    """Batches take cost(group, batch) seconds of the fake clock; a stream runs
    one batch at a time.  fail(group, batch) -> True makes a launch fail."""

    def __init__(self, clock: FakeClock, cost: Callable[[int, int], float], n_streams: int = 2,
                 unit_bytes: int = 1 << 20, ws_bytes: Callable[[int, int], int] = lambda g, b: b << 20,
                 static: int = 0, fail: Callable[[int, int], bool] = lambda g, b: False):
        self.clock, self.cost, self.n_streams = clock, cost, n_streams
        self._ub, self._ws, self._static, self._fail = unit_bytes, ws_bytes, static, fail
        self.busy_until = [0.0] * n_streams
        self.launches: List[Tuple[int, int, int, float]] = []
        self.resident: set = set()

    def admit(self, req):
        self.resident.add(req.rid)

    def release(self, req):
        self.resident.discard(req.rid)

    def unit_bytes(self, group):
        return self._ub

    def static_bytes(self):
        return self._static

    def workspace_bytes(self, group, batch):
        return self._ws(group, batch)

    def launch(self, stream, group, units):
        if self._fail(group, len(units)):
            raise RuntimeError("injected launch failure")
        start = max(self.clock.now(), self.busy_until[stream])
        end = start + self.cost(max(group, 0) if group >= 0 else max(u.group for u in units), len(units))
        self.busy_until[stream] = end
        self.launches.append((stream, group, len(units), start))
        return (end, [("result", u.req.rid, u.group, u.payload) for u in units])

    def done(self, handle):
        return self.clock.now() >= handle[0]

    def next_done_time(self):
        pending = [t for t in self.busy_until if t > self.clock.now()]
        return min(pending) if pending else None

    def results(self, handle):
        return handle[1]


class Server:
    def __init__(self, executor: Executor, clock, n_groups: int, hbm_budget: int, max_batch: int = 16,
                 admit_timeout: float = 10.0, max_queue: int = 100000, mix_groups: bool = False):
        self.ex, self.clock = executor, clock
        self.mix_groups = mix_groups
        self.n_groups, self.max_batch = n_groups, max_batch
        self.budget = hbm_budget
        self.admit_timeout, self.max_queue = admit_timeout, max_queue
        self.waiting: Deque[Request] = collections.deque()
        self.queues: List[Deque[Unit]] = [collections.deque() for _ in range(n_groups)]
        self.free_streams = list(range(executor.n_streams))
        self.running: List[Tuple[int, Any, List[Unit]]] = []
        self.in_flight = 0
        # every stream may hold a workspace for a full batch of the largest group
        # (or, mixing groups, for a full batch over every group's plan)
        if mix_groups:
            self.ws_reserved = executor.n_streams * executor.workspace_bytes(-1, max_batch)
        else:
            self.ws_reserved = executor.n_streams * max(executor.workspace_bytes(g, max_batch)
                                                        for g in range(n_groups))
        self.completed: List[Request] = []
        self.rejected: List[Request] = []
        self.expired: List[Request] = []
        self.cancelled: List[Request] = []
        self.admitted: Dict[int, Request] = {}
        self.failed_batches = 0
        self.batch_sizes: List[int] = []

    # ------------------------------------------------------------------ admission
    def capacity(self) -> int:
        return self.budget - self.ex.static_bytes() - self.ws_reserved

    def submit(self, req: Request) -> bool:
        req.remaining = len(req.units)
        req.bytes_in_flight = sum(2 * self.ex.unit_bytes(g) for g, _ in req.units)
        if req.bytes_in_flight > self.capacity() or len(self.waiting) >= self.max_queue:
            req.rejected = True
            self.rejected.append(req)
            return False
        self.waiting.append(req)
        return True

    def _admit(self, now: float):
        while self.waiting:
            r = self.waiting[0]
            if r.closed:
                self.waiting.popleft()
                continue
            if now - r.arrival > self.admit_timeout:
                self.waiting.popleft()
                r.rejected = True
                self.rejected.append(r)
                continue
            if self.in_flight + r.bytes_in_flight > self.capacity():
                break
            self.waiting.popleft()
            self.in_flight += r.bytes_in_flight
            r.admitted_at = now
            self.admitted[r.rid] = r
            self.ex.admit(r)
            for g, payload in r.units:
                self.queues[g].append(Unit(r, g, payload, now))

    # ------------------------------------------------------------------ cancellation
    def _close(self, r: Request, why: str) -> None:
        """Cancel r: drop its queued units and release its device bytes now;
        units already launched finish and their results are discarded."""
        if r.closed or r.done_at is not None:
            return
        r.cancelled = why
        (self.expired if why == "deadline" else self.cancelled).append(r)
        if self.admitted.pop(r.rid, None) is not None:
            self.in_flight -= r.bytes_in_flight
            self.ex.release(r)
            for q in self.queues:
                if any(u.req is r for u in q):
                    kept = [u for u in q if u.req is not r]
                    q.clear()
                    q.extend(kept)

    def cancel(self, rid: int) -> bool:
        """Client cancellation of a request that has not completed."""
        for r in list(self.waiting) + list(self.admitted.values()):
            if r.rid == rid and not r.closed and r.done_at is None:
                self._close(r, "client")
                return True
        return False

    def _expire(self, now: float) -> None:
        for r in list(self.waiting) + list(self.admitted.values()):
            if r.deadline is not None and not r.closed and now - r.arrival > r.deadline:
                self._close(r, "deadline")

    # ------------------------------------------------------------------ completion
    def _finish(self, now: float):
        still = []
        for stream, handle, units in self.running:
            if self.ex.done(handle):
                outs = self.ex.results(handle)
                for u, o in zip(units, outs):
                    if u.req.closed:
                        continue
                    u.req.results[u.group] = o
                    u.req.remaining -= 1
                    if u.req.remaining == 0:
                        u.req.done_at = self.clock.now()
                        self.in_flight -= u.req.bytes_in_flight
                        self.admitted.pop(u.req.rid, None)
                        self.ex.release(u.req)
                        self.completed.append(u.req)
                self.free_streams.append(stream)
            else:
                still.append((stream, handle, units))
        self.running = still

    # ------------------------------------------------------------------ dispatch
    def _take(self) -> Tuple[int, List[Unit]]:
        """The next batch: up to max_batch units of the group whose oldest unit
        has waited longest, or (mixing groups) the max_batch oldest units of
        any groups, which one launch runs over their different plans."""
        if not self.mix_groups:
            _, g = min((q[0].enq, g) for g, q in enumerate(self.queues) if q)
            q = self.queues[g]
            return g, [q.popleft() for _ in range(min(self.max_batch, len(q)))]
        units: List[Unit] = []
        while len(units) < self.max_batch:
            cands = [(q[0].enq, g) for g, q in enumerate(self.queues) if q]
            if not cands:
                break
            units.append(self.queues[min(cands)[1]].popleft())
        return (units[0].group if len({u.group for u in units}) == 1 else -1), units

    def _dispatch(self, now: float):
        while self.free_streams:
            if not any(self.queues):
                return
            g, units = self._take()
            stream = self.free_streams.pop(0)
            try:
                handle = self.ex.launch(stream, g, units)
            except Exception:
                # the batch's requests fail; the loop continues
                self.failed_batches += 1
                self.free_streams.append(stream)
                for u in units:
                    if not u.req.closed:
                        u.req.rejected = True
                        self.in_flight -= u.req.bytes_in_flight
                        self.admitted.pop(u.req.rid, None)
                        self.ex.release(u.req)
                        self.rejected.append(u.req)
                for qq in self.queues:
                    kept = [u for u in qq if not u.req.closed]
                    qq.clear()
                    qq.extend(kept)
                continue
            self.batch_sizes.append(len(units))
            self.running.append((stream, handle, units))

    def step(self):
        now = self.clock.now()
        self._finish(now)
        self._expire(now)
        self._admit(now)
        self._dispatch(now)

    def idle(self) -> bool:
        return not any(not r.closed for r in self.waiting) and not self.running and not any(self.queues)

    def run(self, requests: Sequence[Request]) -> Dict:
        """Feed requests at their arrival times (seconds after the call) and run
        until all finish.  The requests are consumed: each one's arrival is
        moved onto the server clock and its results, times and state are
        filled in, so a second run takes fresh Request objects."""
        pending = sorted(requests, key=lambda r: r.arrival)
        i = 0
        t0 = self.clock.now()
        while i < len(pending) or not self.idle():
            now = self.clock.now() - t0
            while i < len(pending) and pending[i].arrival <= now:
                pending[i].arrival += t0
                self.submit(pending[i])
                i += 1
            self.step()
            nxt = []
            if i < len(pending):
                nxt.append(t0 + pending[i].arrival)
            nd = self.ex.next_done_time()
            if nd is not None:
                nxt.append(nd)
            dl = [r.arrival + r.deadline for r in list(self.waiting) + list(self.admitted.values())
                  if r.deadline is not None and not r.closed]
            if dl:
                nxt.append(min(dl) + 1e-9)
            if nxt:
                self.clock.sleep_until(min(nxt))
            elif self.running:
                self.clock.sleep_until(self.clock.now() + 2e-4)
            elif self.idle() and i >= len(pending):
                break
        return self.report()

    def report(self) -> Dict:
        lat = np.array([r.latency for r in self.completed]) if self.completed else np.zeros(0)
        if len(self.completed):
            span = max(r.done_at for r in self.completed) - min(r.arrival for r in self.completed)
        else:
            span = 0.0
        units = sum(len(r.units) for r in self.completed)
        return {
            "completed": len(self.completed),
            "rejected": len(self.rejected),
            "expired": len(self.expired),
            "cancelled": len(self.cancelled),
            "failed_batches": self.failed_batches,
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
            "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "units_per_s": units / span if span > 0 else 0.0,
            "span_s": span,
        }


class GpuExecutor(Executor):
    """Runs batches of group selectors through helrm_lookup_packed on HIP
    streams.  Selectors arrive as pinned host tensors; at admission they are
    copied into device memory (a copy stream; the request's in-flight bytes
    are then real HBM), each launch gathers its batch from there, runs the
    lookup and copies the results back, all on its stream; completion or
    cancellation frees the request's device copies."""

    def __init__(self, ctx, plans: Sequence, level: int, N: int, n_streams: int = 2, max_batch: int = 16,
                 static_bytes: int = 0):
        import torch
        self.torch = torch
        self.ctx, self.plans, self.level, self.N = ctx, list(plans), level, N
        self.n_streams = n_streams
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.copy_stream = torch.cuda.Stream()
        self.max_batch = max_batch
        ct_words = 2 * (level + 1) * N
        out_words = 2 * level * N
        self.in_buf = [torch.empty(max_batch, ct_words, dtype=torch.int64, device="cuda") for _ in range(n_streams)]
        self.out_buf = [torch.empty(max_batch, out_words, dtype=torch.int64, device="cuda")
                        for _ in range(n_streams)]
        self.host_out = [torch.empty(max_batch, out_words, dtype=torch.int64, pin_memory=True)
                         for _ in range(n_streams)]
        # keys and plans (given) plus the per-stream staging buffers
        self._static = static_bytes + 8 * n_streams * max_batch * (ct_words + out_words)
        self.resident: Dict[Tuple[int, int], Tuple[Any, Any]] = {}   # (rid, group) -> (device copy, ready event)
        # a full batch over every group's plan bounds any mixed batch's workspace
        self.mix_plans = [self.plans[k % len(self.plans)] for k in range(max_batch)]
        for s in range(n_streams):
            for p in self.plans:
                ctx.helrm_reserve(p, max_batch, self.streams[s])
            ctx.helrm_reserve_batch(self.mix_plans, self.streams[s])

    def close(self):
        """Wait for this executor's streams and give their workspaces back to
        the library (an executor that is replaced by another would otherwise
        leave them allocated until the context is destroyed)."""
        for st in self.streams:
            st.synchronize()
            self.ctx.helrm_release_stream(st)
        self.resident.clear()

    def admit(self, req):
        torch = self.torch
        with torch.cuda.stream(self.copy_stream):
            for g, payload in req.units:
                d = torch.empty(payload.numel(), dtype=torch.int64, device="cuda")
                d.copy_(payload.reshape(-1), non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(self.copy_stream)
                self.resident[(req.rid, g)] = (d, ev)

    def release(self, req):
        for g, _ in req.units:
            self.resident.pop((req.rid, g), None)

    def unit_bytes(self, group):
        return 8 * 2 * (self.level + 1) * self.N

    def static_bytes(self):
        return self._static

    def workspace_bytes(self, group, batch):
        if group < 0:
            return self.ctx.helrm_footprint_batch([self.plans[k % len(self.plans)] for k in range(batch)])
        return self.ctx.helrm_footprint(self.plans[group], batch)

    def launch(self, stream, group, units):
        torch = self.torch
        s = self.streams[stream]
        B = len(units)
        with torch.cuda.stream(s):
            for k, u in enumerate(units):
                res = self.resident.get((u.req.rid, u.group)) if u.req is not None else None
                if res is not None:
                    d, ev = res
                    s.wait_event(ev)
                    self.in_buf[stream][k].copy_(d, non_blocking=True)
                    d.record_stream(s)
                else:
                    self.in_buf[stream][k].copy_(u.payload.reshape(-1), non_blocking=True)
            sel = self.in_buf[stream][:B]
            out = self.out_buf[stream][:B]
            if group >= 0:
                self.ctx.helrm_lookup_packed(self.plans[group], sel, B, out, s)
            else:   # units of several groups: one launch over their plans
                self.ctx.helrm_lookup_batch([self.plans[u.group] for u in units], sel, out, s)
            self.host_out[stream][:B].copy_(out, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, stream, B)

    def done(self, handle):
        return handle[0].query()

    def next_done_time(self):
        return None

    def results(self, handle):
        _, stream, B = handle
        return [self.host_out[stream][k].clone() for k in range(B)]
