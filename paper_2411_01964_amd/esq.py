"""Python binding of libesq (ctypes).  Argument marshalling only: every step of
the computation runs in the HIP kernels behind the C-ABI of include/esq.h.
PyTorch provides device memory and streams.

There is no CPU fallback: if libesq.so has not been built, or no GPU is
present, these functions raise.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libesq.so")

ESQ_RECORDS_CAP = 64
ESQ_EXCEPTIONS_CAP_MAX = 16384
ESQ_MAX_HI = 1 << 56
ESQ_NOALLOC_SCRATCH_MAX = 64 << 20
ESQ_CEILINGS = 8
STATUS_TAIL_OVERFLOW = 1
STATUS_BUCKET_OVERFLOW = 2
STATUS_EXCEPTIONS_INCOMPLETE = 4
RECORD_KMAX_LIMIT = 1

# every function declared in include/esq.h
EXPORTS = ("esq_init", "esq_sieve_segment", "esq_verify_range", "esq_verify_range_noalloc",
           "esq_verify_batch",
           "esq_batch_create", "esq_batch_launch", "esq_batch_destroy",
           "esq_scratch_bytes",
           "esq_set_param", "esq_get_param", "esq_profile_take", "esq_phase_take",
           "esq_measure_ceilings",
           "esq_last_error", "esq_shutdown")


class Summary(ctypes.Structure):
    _fields_ = [
        ("n0", ctypes.c_uint64),
        ("n_odd", ctypes.c_uint64),
        ("hist", ctypes.c_uint64 * 65),
        ("ksum", ctypes.c_uint64),
        ("kmax_seen", ctypes.c_uint32),
        ("n_records", ctypes.c_uint32),
        ("n_exceptions", ctypes.c_uint64),
        ("status", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class Record(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("k", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


SUMMARY_BYTES = ctypes.sizeof(Summary)
PER_N_SLAB = 544 << 20   # per-n output slab of a batch: any interval of up to 2^29 odd n fits
RECORD_BYTES = ctypes.sizeof(Record)


def _np_dtypes():
    import numpy as np
    summary = np.dtype([("n0", "<u8"), ("n_odd", "<u8"), ("hist", "<u8", 65), ("ksum", "<u8"),
                        ("kmax_seen", "<u4"), ("n_records", "<u4"), ("n_exceptions", "<u8"),
                        ("status", "<u4"), ("reserved", "<u4")])
    record = np.dtype([("n", "<u8"), ("k", "<u4"), ("flags", "<u4")])
    assert summary.itemsize == SUMMARY_BYTES and record.itemsize == RECORD_BYTES
    return summary, record


SUMMARY_DTYPE, RECORD_DTYPE = _np_dtypes()


class EsqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libesq error %d: %s" % (code, msg))
        self.code = code


_lock = threading.Lock()
_lib = None


def lib():
    """Load libesq.so (raises if it was not built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libesq.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        u64, u32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        L.esq_init.argtypes = [ctypes.c_int, u64]
        L.esq_init.restype = ctypes.c_int
        L.esq_sieve_segment.argtypes = [u64, u64, vp, vp]
        L.esq_sieve_segment.restype = ctypes.c_int
        L.esq_verify_range.argtypes = [u64, u64, u32, vp, vp, vp, vp, u64, vp]
        L.esq_verify_range.restype = ctypes.c_int
        L.esq_verify_range_noalloc.argtypes = [u64, u64, u32, vp, vp, vp, vp, u64, vp]
        L.esq_verify_range_noalloc.restype = ctypes.c_int
        L.esq_verify_batch.argtypes = [u32, vp, vp, u32, vp, vp, vp, vp]
        L.esq_verify_batch.restype = ctypes.c_int
        L.esq_batch_create.argtypes = [u32, vp, vp, u32, vp, vp, vp, ctypes.POINTER(vp)]
        L.esq_batch_create.restype = ctypes.c_int
        L.esq_batch_launch.argtypes = [vp, ctypes.c_int, vp]
        L.esq_batch_launch.restype = ctypes.c_int
        L.esq_batch_destroy.argtypes = [vp]
        L.esq_batch_destroy.restype = None
        L.esq_scratch_bytes.argtypes = [u32, vp, vp, u32, ctypes.POINTER(u64)]
        L.esq_scratch_bytes.restype = ctypes.c_int
        L.esq_set_param.argtypes = [ctypes.c_char_p, ctypes.c_int64]
        L.esq_set_param.restype = ctypes.c_int
        L.esq_get_param.argtypes = [ctypes.c_char_p]
        L.esq_get_param.restype = ctypes.c_int64
        L.esq_profile_take.argtypes = [ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_uint64)]
        L.esq_profile_take.restype = ctypes.c_int
        L.esq_phase_take.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
        L.esq_phase_take.restype = ctypes.c_int
        L.esq_measure_ceilings.argtypes = [ctypes.POINTER(ctypes.c_double)]
        L.esq_measure_ceilings.restype = ctypes.c_int
        L.esq_last_error.restype = ctypes.c_char_p
        L.esq_shutdown.restype = None
        _lib = L
        return L


def _check(rc):
    if rc != 0:
        raise EsqError(rc, lib().esq_last_error().decode())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _per_n_buffer(n0: int, n_odd: int, dev):
    """Device bytes for the per-n output of the odd n from n0: a view placed
    so that its address is congruent to n0's odd index mod 16.  The library
    writes each wave's 4 KB run of bytes with 16-byte stores from 16-byte
    boundaries then, without the shifted path for a misaligned run."""
    buf = torch.empty(max(n_odd, 1) + 16, dtype=torch.uint8, device=dev)
    off = (((n0 - 1) // 2) - buf.data_ptr()) % 16
    return buf[off:off + max(n_odd, 1)]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def init(device: int = 0, max_hi: int = (1 << 50) + (1 << 32)):
    """Make the library resident on `device` for ranges up to max_hi."""
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: libesq runs on the GPU only")
    torch.cuda.set_device(device)
    _check(lib().esq_init(int(device), int(max_hi)))


def shutdown():
    lib().esq_shutdown()


def set_param(name: str, value: int):
    _check(lib().esq_set_param(name.encode(), int(value)))


def get_param(name: str) -> int:
    return int(lib().esq_get_param(name.encode()))


def scratch_bytes(los, his, kmax: int = 0) -> int:
    """Device scratch (bytes) that one esq_verify_batch call over these
    intervals takes from the library's pool while it runs (esq_scratch_bytes);
    the caller's outputs are not included."""
    import numpy as np
    lo = np.ascontiguousarray(np.asarray(los, dtype=np.uint64))
    hi = np.ascontiguousarray(np.asarray(his, dtype=np.uint64))
    out = ctypes.c_uint64(0)
    _check(lib().esq_scratch_bytes(int(lo.size), ctypes.c_void_p(lo.ctypes.data),
                                   ctypes.c_void_p(hi.ctypes.data), int(kmax), ctypes.byref(out)))
    return int(out.value)


def profile_take():
    """(total_ms, launches) of segment-kernel launches recorded while the knob
    "profile" was 1, since the previous take."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_uint64(0)
    _check(lib().esq_profile_take(ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


def phase_take() -> dict:
    """Segment-kernel time per phase, summed over workgroups, in ticks of the
    device's constant-rate counter, while "phase_clock" was 1, since the
    previous take."""
    out = (ctypes.c_uint64 * 3)()
    _check(lib().esq_phase_take(out))
    return {"init": int(out[0]), "mark": int(out[1]), "search_or_store": int(out[2])}


def measure_ceilings() -> dict:
    """Measured LDS, VALU, L2 and HBM-write ceilings of the current device
    (microbenchmarks): bytes/s of conflict-free ds_write_b64, ds_read_b64,
    ds_or_b32, int32 VALU lane-operations/s of full-rate adds/xors, funnel
    shifts and popcounts, bytes/s of 16-byte L2 reads, and bytes/s of
    16-byte stores streaming to HBM."""
    out = (ctypes.c_double * ESQ_CEILINGS)()
    _check(lib().esq_measure_ceilings(out))
    return {"lds_write_b64_Bps": out[0], "lds_read_b64_Bps": out[1], "lds_or_b32_Bps": out[2],
            "valu_int32_ops_per_s": out[3], "valu_alignbit_ops_per_s": out[4],
            "valu_bcnt_ops_per_s": out[5], "l2_read_Bps": out[6],
            "hbm_write_Bps": out[7]}


def sieve_segment(lo: int, hi: int, out=None, stream=None):
    """Algorithm 1 alone on the odd m in [lo, hi).  Returns (m0, n_bits,
    words) with `words` an int64 device tensor holding the little-endian
    uint64 bit stream (bit i set iff m0 + 2i is squarefree)."""
    lo, hi = int(lo), int(hi)
    m0 = max(lo, 1) | 1
    n = (hi - m0 + 1) // 2 if hi > m0 else 0
    nw = (n + 63) // 64
    if out is None:
        out = torch.empty(max(nw, 1), dtype=torch.int64, device="cuda")
    elif out.numel() < nw or out.dtype != torch.int64 or not out.is_cuda:
        raise ValueError("out must be an int64 CUDA tensor of >= %d words" % nw)
    _check(lib().esq_sieve_segment(lo, hi, _ptr(out), _stream(stream)))
    return m0, n, out[:nw]


class Pending:
    """Device buffers of one enqueued esq_verify_range call."""

    def __init__(self, lo, hi, kmax, per_n, exceptions_cap, stream, noalloc=False):
        self.lo, self.hi, self.kmax = int(lo), int(hi), int(kmax)
        n0 = max(self.lo, 3) | 1
        self.n_odd = (self.hi - n0 + 1) // 2 if self.hi > n0 else 0
        dev = torch.device("cuda", torch.cuda.current_device())
        self.summary = torch.empty(SUMMARY_BYTES, dtype=torch.uint8, device=dev)
        self.records = torch.empty(ESQ_RECORDS_CAP * RECORD_BYTES, dtype=torch.uint8, device=dev)
        self.exc_cap = int(exceptions_cap)
        self.exceptions = (torch.empty(self.exc_cap, dtype=torch.int64, device=dev)
                           if self.exc_cap else None)
        self.per_n = _per_n_buffer(n0, self.n_odd, dev) if per_n else None
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        call = lib().esq_verify_range_noalloc if noalloc else lib().esq_verify_range
        _check(call(
            self.lo, self.hi, self.kmax, _ptr(self.per_n), _ptr(self.summary),
            _ptr(self.records), _ptr(self.exceptions), self.exc_cap,
            ctypes.c_void_p(self.stream.cuda_stream)))
        self.event = torch.cuda.Event()
        self.event.record(self.stream)

    def done(self) -> bool:
        return self.event.query()

    def result(self, check: bool = True) -> dict:
        self.event.synchronize()
        s = Summary.from_buffer_copy(bytes(self.summary.cpu().numpy().tobytes()))
        recs_raw = self.records.cpu().numpy().tobytes()
        nrec = min(s.n_records, ESQ_RECORDS_CAP)
        recs, flags = [], []
        for i in range(nrec):
            r = Record.from_buffer_copy(recs_raw[i * RECORD_BYTES:(i + 1) * RECORD_BYTES])
            recs.append((int(r.n), int(r.k)))
            flags.append(int(r.flags))
        nexc = min(int(s.n_exceptions), self.exc_cap)
        exc = [int(x) for x in self.exceptions[:nexc].cpu().tolist()] if nexc else []
        out = {
            "n0": int(s.n0),
            "n_odd": int(s.n_odd),
            "hist": [int(x) for x in s.hist],
            "ksum": int(s.ksum),
            "kmax_seen": int(s.kmax_seen),
            "n_records": int(s.n_records),
            "records": recs,
            "record_flags": flags,
            "n_exceptions": int(s.n_exceptions),
            "exceptions": exc,
            "status": int(s.status),
        }
        if self.per_n is not None:
            out["per_n"] = self.per_n[:self.n_odd]
        if check and s.status:
            raise EsqError(-100, "device status 0x%x for [%d, %d)" % (s.status, self.lo, self.hi))
        return out


def verify_range_async(lo, hi, kmax=0, per_n=False, exceptions_cap=0, stream=None,
                       noalloc=False) -> Pending:
    """Enqueue Algorithm 2 over the odd n in [lo, hi); returns a Pending.
    noalloc=True goes through esq_verify_range_noalloc (the library's static
    scratch; calls on one device must not overlap)."""
    return Pending(lo, hi, kmax, per_n, exceptions_cap, stream, noalloc)


def verify_range(lo, hi, kmax=0, per_n=False, exceptions_cap=0, stream=None, check=True,
                 noalloc=False) -> dict:
    """Algorithm 2 over every odd n >= 3 in [lo, hi) plus the aggregates
    (per-k counts, sum of k, maximum k, record-setters, exceptions).  With
    per_n=True the result holds "per_n", a uint8 CUDA tensor of least k."""
    return verify_range_async(lo, hi, kmax, per_n, exceptions_cap, stream,
                              noalloc).result(check=check)


def _parse(summary_bytes, record_bytes):
    s = Summary.from_buffer_copy(summary_bytes)
    nrec = min(s.n_records, ESQ_RECORDS_CAP)
    recs, flags = [], []
    for i in range(nrec):
        r = Record.from_buffer_copy(record_bytes[i * RECORD_BYTES:(i + 1) * RECORD_BYTES])
        recs.append((int(r.n), int(r.k)))
        flags.append(int(r.flags))
    return {
        "n0": int(s.n0),
        "n_odd": int(s.n_odd),
        "hist": [int(x) for x in s.hist],
        "ksum": int(s.ksum),
        "kmax_seen": int(s.kmax_seen),
        "n_records": int(s.n_records),
        "records": recs,
        "record_flags": flags,
        "n_exceptions": int(s.n_exceptions),
        "status": int(s.status),
    }


def _parse_many(summaries, records, count):
    """Summaries and records of count intervals from their device buffers."""
    sm = summaries[:count * SUMMARY_BYTES].cpu().numpy().view(SUMMARY_DTYPE)
    rc = records[:count * ESQ_RECORDS_CAP * RECORD_BYTES].cpu().numpy().view(RECORD_DTYPE)
    rc = rc.reshape(count, ESQ_RECORDS_CAP)
    hist = sm["hist"].tolist()
    cols = {k: sm[k].tolist() for k in ("n0", "n_odd", "ksum", "kmax_seen", "n_records",
                                         "n_exceptions", "status")}
    rn, rk, rf = rc["n"].tolist(), rc["k"].tolist(), rc["flags"].tolist()
    out = []
    for i in range(count):
        nrec = min(cols["n_records"][i], ESQ_RECORDS_CAP)
        out.append({
            "n0": cols["n0"][i], "n_odd": cols["n_odd"][i], "hist": hist[i],
            "ksum": cols["ksum"][i], "kmax_seen": cols["kmax_seen"][i],
            "n_records": cols["n_records"][i],
            "records": list(zip(rn[i][:nrec], rk[i][:nrec])),
            "record_flags": rf[i][:nrec],
            "n_exceptions": cols["n_exceptions"][i], "status": cols["status"][i],
        })
    return out


class PendingBatch:
    """Device buffers of one enqueued esq_verify_batch call."""

    def __init__(self, los, his, kmax, per_n, stream, host_bufs=None, alloc_stream=None):
        import numpy as np
        self.lo = np.ascontiguousarray(np.asarray(los, dtype=np.uint64))
        self.hi = np.ascontiguousarray(np.asarray(his, dtype=np.uint64))
        if self.lo.shape != self.hi.shape or self.lo.ndim != 1:
            raise ValueError("lo and hi must be 1-D of equal length")
        self.count = int(self.lo.size)
        dev = torch.device("cuda", torch.cuda.current_device())
        self.summaries = torch.empty(max(self.count, 1) * SUMMARY_BYTES, dtype=torch.uint8, device=dev)
        self.records = torch.empty(max(self.count, 1) * ESQ_RECORDS_CAP * RECORD_BYTES,
                                   dtype=torch.uint8, device=dev)
        self.per_n = None
        ptrs = None
        if per_n is not None and any(per_n):
            # per-n outputs packed into slabs of one fixed size (a size the
            # caching allocator hands out again and again), a larger output in
            # an allocation of its own; each interval's bytes start at an
            # address congruent to its first odd index mod 16 (as
            # _per_n_buffer places a single one)
            lo_l, hi_l = self.lo.tolist(), self.hi.tolist()
            self.per_n = [None] * self.count
            ptrs = (ctypes.c_void_p * self.count)()
            buf, base, off, cap = None, 0, 0, 0
            for i in range(self.count):
                if not per_n[i]:
                    continue
                n0 = max(lo_l[i], 3) | 1
                n = (hi_l[i] - n0 + 1) // 2 if hi_l[i] > n0 else 0
                need = max(n, 1) + 15
                if buf is None or off + need > cap:
                    cap = max(PER_N_SLAB, need)
                    if alloc_stream is None:
                        buf = torch.empty(cap, dtype=torch.uint8, device=dev)
                    else:
                        # from one stream's pool whichever stream runs the batch
                        # (the caching allocator reuses a block only on the
                        # stream it was allocated on); recorded on the batch's
                        # stream so that it is not reused before the batch ends
                        with torch.cuda.stream(alloc_stream):
                            buf = torch.empty(cap, dtype=torch.uint8, device=dev)
                        buf.record_stream(stream if stream is not None else torch.cuda.current_stream())
                    base, off = buf.data_ptr(), 0
                off += (((n0 - 1) // 2) - (base + off)) % 16
                self.per_n[i] = buf[off:off + n]
                ptrs[i] = base + off
                off += max(n, 1)
            del buf
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().esq_verify_batch(
            self.count, ctypes.c_void_p(self.lo.ctypes.data), ctypes.c_void_p(self.hi.ctypes.data),
            int(kmax), ptrs, _ptr(self.summaries), _ptr(self.records),
            ctypes.c_void_p(self.stream.cuda_stream)))
        # with host_bufs (pinned host tensors the caller reuses for one batch
        # at a time), the summaries and records are copied there on the
        # batch's own stream, so that they are on the host when its event
        # completes
        self.host_bufs = None
        if host_bufs is not None:
            hs, hr = host_bufs
            if hs.numel() < self.summaries.numel() or hr.numel() < self.records.numel():
                raise ValueError("host buffers too small for the batch")
            self.host_bufs = (hs[:self.summaries.numel()], hr[:self.records.numel()])
            with torch.cuda.stream(self.stream):
                self.host_bufs[0].copy_(self.summaries, non_blocking=True)
                self.host_bufs[1].copy_(self.records, non_blocking=True)
        self.event = torch.cuda.Event()
        self.event.record(self.stream)

    def done(self) -> bool:
        return self.event.query()

    def result(self, check: bool = True) -> list:
        self.event.synchronize()
        out = _parse_many(self.summaries, self.records, self.count)
        for i, r in enumerate(out):
            if self.per_n is not None and self.per_n[i] is not None:
                r["per_n"] = self.per_n[i]
            if check and r["status"]:
                raise EsqError(-100, "device status 0x%x for interval %d" % (r["status"], i))
        return out

    def raw(self, check: bool = True) -> "BatchResults":
        """The batch's results as arrays, parsed per interval on demand (a
        copy of the host buffers when the batch was given some, so that they
        can take the next batch)."""
        self.event.synchronize()
        if self.host_bufs is not None:
            return BatchResults(self.host_bufs[0], self.host_bufs[1], self.count, self.per_n, check,
                                copy=True)
        return BatchResults(self.summaries, self.records, self.count, self.per_n, check)


class BatchResults:
    """Summaries and records of a batch copied to the host in two transfers;
    interval i becomes the dict of verify_range only when asked for."""

    def __init__(self, summaries, records, count, per_n, check, copy=False):
        import numpy as np
        self.count = count
        sm = summaries[:count * SUMMARY_BYTES].cpu().numpy()
        rc = records[:count * ESQ_RECORDS_CAP * RECORD_BYTES].cpu().numpy()
        if copy:
            sm, rc = np.array(sm), np.array(rc)
        self.sm = sm.view(SUMMARY_DTYPE)
        self.rc = rc.view(RECORD_DTYPE).reshape(count, ESQ_RECORDS_CAP)
        self.per_n = per_n
        if check and count and self.sm["status"].any():
            i = int(self.sm["status"].nonzero()[0][0])
            raise EsqError(-100, "device status 0x%x for interval %d" % (int(self.sm["status"][i]), i))

    def release_per_n(self, i):
        """Drop the batch's reference to interval i's per-n bytes."""
        if self.per_n is not None:
            self.per_n[i] = None

    def parse(self, i) -> dict:
        s, rc = self.sm[i], self.rc[i]
        nrec = min(int(s["n_records"]), ESQ_RECORDS_CAP)
        out = {
            "n0": int(s["n0"]), "n_odd": int(s["n_odd"]), "hist": s["hist"].tolist(),
            "ksum": int(s["ksum"]), "kmax_seen": int(s["kmax_seen"]),
            "n_records": int(s["n_records"]),
            "records": list(zip(rc["n"][:nrec].tolist(), rc["k"][:nrec].tolist())),
            "record_flags": rc["flags"][:nrec].tolist(),
            "n_exceptions": int(s["n_exceptions"]), "status": int(s["status"]),
        }
        if self.per_n is not None and self.per_n[i] is not None:
            out["per_n"] = self.per_n[i]
        return out


def verify_batch_async(los, his, kmax=0, per_n=None, stream=None, host_bufs=None,
                       alloc_stream=None) -> PendingBatch:
    """Enqueue many intervals in one launch (esq_verify_batch)."""
    return PendingBatch(los, his, kmax, per_n, stream, host_bufs, alloc_stream)


def verify_batch(los, his, kmax=0, per_n=None, stream=None, check=True) -> list:
    """Per-interval results of esq_verify_batch, in input order."""
    return verify_batch_async(los, his, kmax, per_n, stream).result(check=check)


class PreparedBatch:
    """A batch planned once (esq_batch_create) and launched many times, as
    plain launches or as a replayed hipGraph (esq_batch_launch)."""

    def __init__(self, los, his, kmax=0):
        import numpy as np
        self.lo = np.ascontiguousarray(np.asarray(los, dtype=np.uint64))
        self.hi = np.ascontiguousarray(np.asarray(his, dtype=np.uint64))
        self.count = int(self.lo.size)
        dev = torch.device("cuda", torch.cuda.current_device())
        self.summaries = torch.empty(self.count * SUMMARY_BYTES, dtype=torch.uint8, device=dev)
        self.records = torch.empty(self.count * ESQ_RECORDS_CAP * RECORD_BYTES,
                                   dtype=torch.uint8, device=dev)
        h = ctypes.c_void_p(None)
        _check(lib().esq_batch_create(self.count, ctypes.c_void_p(self.lo.ctypes.data),
                                      ctypes.c_void_p(self.hi.ctypes.data), int(kmax), None,
                                      _ptr(self.summaries), _ptr(self.records), ctypes.byref(h)))
        self.handle = h

    def launch(self, graph=False, stream=None):
        _check(lib().esq_batch_launch(self.handle, 1 if graph else 0, _stream(stream)))

    def results(self, check=True):
        torch.cuda.synchronize()
        out = _parse_many(self.summaries, self.records, self.count)
        for i, r in enumerate(out):
            if check and r["status"]:
                raise EsqError(-100, "device status 0x%x for interval %d" % (r["status"], i))
        return out

    def close(self):
        if self.handle:
            lib().esq_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
