"""Serving: continuous batching of interval-verification requests.

Requests (an interval [lo, hi) and whether the per-n least k is wanted)
arrive at any time.  A scheduler thread admits waiting requests into a batch
whenever a stream slot is free and the batch's HBM footprint fits the budget,
and launches the batch with one esq_verify_batch call (one persistent kernel
over a device work queue).  Batches on different streams overlap on the
device, so requests that arrive while others run are admitted as soon as a
slot and memory free up.  The prime table and the wheel pattern stay resident
in the library's context; a batch's scratch is stream-ordered.

Results are exactly those of esq_verify_range on each interval alone (the
tests check this); only latency and throughput depend on the mix.
"""
from __future__ import annotations

import collections
import gc
import threading
import time

import torch

from . import esq

# scratch bytes a batch needs per odd n besides the per-n output (hit slots,
# counters), a conservative figure for sizing admission
_SCRATCH_PER_N = 0.01
_SCRATCH_PER_REQUEST = 64 << 10


def footprint(lo: int, hi: int, per_n: bool) -> int:
    """HBM bytes a request holds while in flight."""
    n0 = max(int(lo), 3) | 1
    n = (int(hi) - n0 + 1) // 2 if int(hi) > n0 else 0
    return int(n * _SCRATCH_PER_N) + _SCRATCH_PER_REQUEST + (n if per_n else 0)


_gc_lock = threading.Lock()
_gc_state = {"servers": 0, "was_enabled": True}


def _gc_pause():
    with _gc_lock:
        if _gc_state["servers"] == 0:
            _gc_state["was_enabled"] = gc.isenabled()
            gc.freeze()
            gc.disable()
        _gc_state["servers"] += 1


def _gc_resume():
    with _gc_lock:
        _gc_state["servers"] -= 1
        if _gc_state["servers"] == 0:
            gc.unfreeze()
            if _gc_state["was_enabled"]:
                gc.enable()


class Request:
    __slots__ = ("lo", "hi", "per_n", "t_arrival", "t_done", "result", "event", "bytes")

    def __init__(self, lo, hi, per_n, t_arrival):
        self.lo, self.hi, self.per_n = int(lo), int(hi), bool(per_n)
        self.t_arrival = t_arrival
        self.t_done = None
        self.result = None
        self.event = threading.Event()
        self.bytes = footprint(lo, hi, per_n)

    def wait(self, timeout=None):
        self.event.wait(timeout)
        return self.result


class Server:
    """Continuous-batching server over the batched C-ABI call."""

    def __init__(self, n_streams: int = 4, hbm_budget: int = 16 << 30, max_batch: int = 512,
                 kmax: int = 0, on_done=None, pause_gc: bool = True, poll_s: float = 0.0):
        # Python's cyclic garbage collector stops every thread while it scans
        # the heap: with tens of thousands of requests alive, a full pass takes
        # 30-150 ms and lands on whichever requests are in flight (it set the
        # p99 latency).  Requests and results form no reference cycles, so
        # reference counting frees them; the collector is paused (and the
        # objects alive at start frozen) while the server runs, and restored
        # by close().
        self._gc_paused = False
        if pause_gc:
            _gc_pause()
            self._gc_paused = True
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.busy = [None] * n_streams          # (PendingBatch, [Request]) per stream
        self.budget = int(hbm_budget)
        self.in_flight_bytes = 0
        self.max_batch = int(max_batch)
        self.kmax = int(kmax)
        self.waiting = collections.deque()
        self.cv = threading.Condition()
        self.running = True
        self.batches = 0
        self.error = None
        self.on_done = on_done
        # how long the scheduler sleeps between completion checks while
        # batches are in flight (HIP events are polled, not waited on).  0:
        # it spins, which halves the median latency of the Poisson stream
        # (0.42 -> 0.19 ms, p99 0.87 -> 0.60 ms) for one busy host core while
        # work is in flight; when idle it sleeps on the condition variable.
        self.poll_s = float(poll_s)
        self.thread = threading.Thread(target=self._loop, name="esq-serve", daemon=True)
        self.thread.start()

    def submit(self, lo, hi, per_n=False) -> Request:
        r = Request(lo, hi, per_n, time.perf_counter())
        with self.cv:
            if self.error is not None:
                raise self.error
            self.waiting.append(r)
            self.cv.notify()
        return r

    def close(self):
        with self.cv:
            self.running = False
            self.cv.notify()
        self.thread.join()
        if self._gc_paused:
            _gc_resume()
            self._gc_paused = False
        if self.error is not None:
            raise self.error

    # ------------------------------------------------------------ scheduler
    def _complete(self, i):
        pend, reqs = self.busy[i]
        res = pend.result(check=True)
        now = time.perf_counter()
        for r, x in zip(reqs, res):
            r.result = x
            r.t_done = now
            self.in_flight_bytes -= r.bytes
            if self.on_done is not None:
                self.on_done(r)
            r.event.set()
        self.busy[i] = None

    def _admit(self, i):
        batch, total = [], 0
        while self.waiting and len(batch) < self.max_batch:
            r = self.waiting[0]
            if batch and self.in_flight_bytes + total + r.bytes > self.budget:
                break
            if not batch and self.in_flight_bytes + r.bytes > self.budget and any(self.busy):
                break  # wait for memory to free up
            batch.append(self.waiting.popleft())
            total += r.bytes
        if not batch:
            return False
        self.in_flight_bytes += total
        with torch.cuda.stream(self.streams[i]):
            pend = esq.verify_batch_async([r.lo for r in batch], [r.hi for r in batch],
                                          kmax=self.kmax, per_n=[r.per_n for r in batch],
                                          stream=self.streams[i])
        self.busy[i] = (pend, batch)
        self.batches += 1
        return True

    def _loop(self):
        try:
            while True:
                progressed = False
                for i, b in enumerate(self.busy):
                    if b is not None and b[0].done():
                        self._complete(i)
                        progressed = True
                with self.cv:
                    if not self.running and not self.waiting and not any(self.busy):
                        return
                    for i in range(len(self.streams)):
                        if self.busy[i] is None and self.waiting:
                            progressed |= self._admit(i)
                    if not progressed:
                        if any(self.busy):
                            self.cv.wait(timeout=self.poll_s)
                        else:
                            self.cv.wait(timeout=0.01)
        except Exception as e:  # surfaced to submitters and close()
            self.error = e
            with self.cv:
                while self.waiting:
                    r = self.waiting.popleft()
                    r.event.set()
            for b in self.busy:
                if b is not None:
                    for r in b[1]:
                        r.event.set()


def _release_per_n(r):
    # the client has consumed the per-n array: give its memory back
    if r.result is not None:
        r.result.pop("per_n", None)


def run_stream(requests, n_streams=4, hbm_budget=16 << 30, warmup_s=1.0, paced=True,
               keep_per_n=True, poll_s=0.0):
    """Drive a Server with (t_arrival_s, lo, hi, per_n) requests.  With
    paced=True each request is submitted at its arrival time; otherwise all
    at once.  With keep_per_n=False per-n arrays are released as soon as each
    request completes.  Returns (list of Request, wall seconds, stats dict)."""
    srv = Server(n_streams=n_streams, hbm_budget=hbm_budget,
                 on_done=None if keep_per_n else _release_per_n, poll_s=poll_s)
    out = []
    t0 = time.perf_counter()
    for t, lo, hi, per_n in requests:
        if paced:
            delay = t - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
        out.append((t, srv.submit(lo, hi, per_n)))
    for _, r in out:
        r.wait()
    wall = time.perf_counter() - t0
    srv.close()
    lat = sorted((r.t_done - r.t_arrival) for t, r in out if t >= warmup_s)
    n_total = sum(r.result["n_odd"] for _, r in out if r.result is not None)
    stats = {
        "requests": len(out),
        "measured_requests": len(lat),
        "batches": srv.batches,
        "p50_ms": 1e3 * lat[len(lat) // 2] if lat else None,
        "p99_ms": 1e3 * lat[min(len(lat) - 1, int(0.99 * len(lat)))] if lat else None,
        "odd_n": n_total,
        "wall_s": wall,
    }
    return [r for _, r in out], wall, stats
