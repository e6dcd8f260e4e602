"""Serving: continuous batching of interval-verification requests.

Requests (an interval [lo, hi) and whether the per-n least k is wanted)
arrive at any time.  A scheduler thread keeps two queues, per-n requests and
summary requests, and whenever a stream slot is free it admits a batch from
the queue whose oldest request has waited longest: one esq_verify_batch call
(one persistent kernel over a device work queue).  Per-n and summary requests
go in separate batches, so summary requests run in the segment kernel's
summary form (twice the resident workgroups of the per-n form, no HBM
writes).  A batch is admitted while its HBM footprint fits the budget: the
scratch the library plans for exactly that batch (esq_scratch_bytes) plus its
outputs.  Batches on different streams overlap on the device, so requests
that arrive while others run are admitted as soon as a slot and memory free
up.  The prime table and the pattern tables stay resident in the library.

Results are exactly those of esq_verify_range on each interval alone (the
tests check this); only latency and throughput depend on the mix.  A
request's result dict is built from the batch's arrays when it is first read.
"""
from __future__ import annotations

import collections
import gc
import threading
import time

import torch

from . import esq

# per-request device bytes besides the per-n output, a planning estimate
# (hit slots and counters per segment of 2^18 odd n, descriptors, outputs);
# the batch's exact scratch comes from the library when it is admitted
_SCRATCH_PER_SEGMENT = 400
_SCRATCH_PER_REQUEST = 4 << 10
_OUTPUT_PER_REQUEST = esq.SUMMARY_BYTES + esq.ESQ_RECORDS_CAP * esq.RECORD_BYTES


def footprint(lo: int, hi: int, per_n: bool) -> int:
    """Estimated HBM bytes a request holds while in flight."""
    n0 = max(int(lo), 3) | 1
    n = (int(hi) - n0 + 1) // 2 if int(hi) > n0 else 0
    return (((n >> 18) + 2) * _SCRATCH_PER_SEGMENT + _SCRATCH_PER_REQUEST +
            _OUTPUT_PER_REQUEST + (n + 16 if per_n else 0))


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
    __slots__ = ("lo", "hi", "per_n", "t_arrival", "t_done", "bytes", "n_odd", "_result", "_src",
                 "_srv")

    def __init__(self, lo, hi, per_n, t_arrival, srv=None):
        self.lo, self.hi, self.per_n = int(lo), int(hi), bool(per_n)
        n0 = max(self.lo, 3) | 1
        self.n_odd = (self.hi - n0 + 1) // 2 if self.hi > n0 else 0
        self.t_arrival = t_arrival
        self.t_done = None
        self.bytes = footprint(lo, hi, per_n)
        self._result = None
        self._src = None          # (BatchResults, index) until the result is read
        self._srv = srv

    @property
    def result(self):
        if self._src is not None:
            batch, i = self._src
            self._src = None
            self._result = batch.parse(i)
        return self._result

    @result.setter
    def result(self, value):
        self._src = None
        self._result = value

    def wait(self, timeout=None):
        """Block until the request is done (or the server failed); returns
        the result dict, or None on a timeout or a server error."""
        if self.t_done is None and self._srv is not None:
            self._srv._wait_done(self, timeout)
        return self.result if self.t_done is not None else None


class Server:
    """Continuous-batching server over the batched C-ABI call."""

    def __init__(self, n_streams: int = 4, hbm_budget: int = 64 << 30, max_batch: int = 512,
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
        # pinned host buffers per stream slot for a batch's summaries and
        # records (copied on the batch's stream, read once it completes)
        self.host_bufs = [(torch.empty(max_batch * esq.SUMMARY_BYTES, dtype=torch.uint8,
                                       pin_memory=True),
                           torch.empty(max_batch * esq.ESQ_RECORDS_CAP * esq.RECORD_BYTES,
                                       dtype=torch.uint8, pin_memory=True))
                          for _ in range(n_streams)]
        self.busy = [None] * n_streams          # (PendingBatch, [Request], bytes) per stream
        self.budget = int(hbm_budget)
        self.in_flight_bytes = 0
        self.max_batch = int(max_batch)
        self.kmax = int(kmax)
        self.queues = (collections.deque(), collections.deque())  # summary, per-n
        self.cv = threading.Condition()
        self.done_cv = threading.Condition()
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
        r = Request(lo, hi, per_n, time.perf_counter(), self)
        with self.cv:
            if self.error is not None:
                raise self.error
            self.queues[1 if r.per_n else 0].append(r)
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

    def _wait_done(self, r, timeout):
        end = None if timeout is None else time.perf_counter() + timeout
        with self.done_cv:
            while r.t_done is None and self.error is None:
                left = None if end is None else end - time.perf_counter()
                if left is not None and left <= 0:
                    return
                self.done_cv.wait(left)

    # ------------------------------------------------------------ scheduler
    def _complete(self, i):
        pend, reqs, nbytes = self.busy[i]
        res = pend.raw(check=True)
        now = time.perf_counter()
        for j, r in enumerate(reqs):
            r._src = (res, j)
            r.t_done = now
            if self.on_done is not None:
                self.on_done(r)
        self.in_flight_bytes -= nbytes
        self.busy[i] = None
        with self.done_cv:
            self.done_cv.notify_all()

    def _admit(self, i):
        qs, qp = self.queues
        if qs and (not qp or qs[0].t_arrival <= qp[0].t_arrival):
            q = qs
        elif qp:
            q = qp
        else:
            return False
        # a batch takes at most its stream's share of the budget, so that
        # several batches are queued on the device while the host completes
        # and admits others (one batch holding the whole budget would leave
        # the GPU idle for every turnaround)
        share = self.budget // len(self.streams)
        batch, total = [], 0
        while q and len(batch) < self.max_batch:
            r = q[0]
            if batch and (self.in_flight_bytes + total + r.bytes > self.budget or
                          total + r.bytes > share):
                break
            if not batch and self.in_flight_bytes + r.bytes > self.budget and any(self.busy):
                break  # wait for memory to free up
            batch.append(q.popleft())
            total += r.bytes
        if not batch:
            return False
        # the library's plan of exactly this batch: its scratch, plus the
        # outputs; a batch that does not fit gives back its last requests
        los, his = [r.lo for r in batch], [r.hi for r in batch]
        while True:
            exact = (esq.scratch_bytes(los, his, self.kmax) + len(batch) * _OUTPUT_PER_REQUEST +
                     sum(r.n_odd + 16 for r in batch if r.per_n))
            if len(batch) == 1 or (self.in_flight_bytes + exact <= self.budget and exact <= share):
                break
            keep = max(1, len(batch) // 2)
            for r in reversed(batch[keep:]):
                q.appendleft(r)
            del batch[keep:], los[keep:], his[keep:]
        if self.in_flight_bytes + exact > self.budget and any(self.busy):
            for r in reversed(batch):
                q.appendleft(r)
            return False
        self.in_flight_bytes += exact
        per_n = batch[0].per_n
        with torch.cuda.stream(self.streams[i]):
            pend = esq.verify_batch_async(los, his, kmax=self.kmax,
                                          per_n=[True] * len(batch) if per_n else None,
                                          stream=self.streams[i], host_bufs=self.host_bufs[i],
                                          alloc_stream=torch.cuda.default_stream())
        self.busy[i] = (pend, batch, exact)
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
                    if (not self.running and not self.queues[0] and not self.queues[1]
                            and not any(self.busy)):
                        return
                    for i in range(len(self.streams)):
                        if self.busy[i] is None and (self.queues[0] or self.queues[1]):
                            progressed |= self._admit(i)
                    if not progressed:
                        if any(self.busy):
                            self.cv.wait(timeout=self.poll_s)
                        else:
                            self.cv.wait(timeout=0.01)
        except Exception as e:  # surfaced to submitters, waiters and close()
            self.error = e
            with self.cv:
                for q in self.queues:
                    q.clear()
            with self.done_cv:
                self.done_cv.notify_all()


def _release_per_n(r):
    # the client has consumed the per-n array: give its memory back
    if r._src is not None:
        r._src[0].release_per_n(r._src[1])
    elif r._result is not None:
        r._result.pop("per_n", None)


def run_stream(requests, n_streams=4, hbm_budget=64 << 30, warmup_s=1.0, paced=True,
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
    n_total = sum(r.n_odd for _, r in out if r.t_done is not None)
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
