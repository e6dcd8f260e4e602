"""ctypes wrapper of the C oracle (test infrastructure only).

Each function restates which part of the paper it follows; the arithmetic
itself lives in ``esq_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "esq_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


class _Summary(ctypes.Structure):
    _fields_ = [
        ("n0", ctypes.c_uint64),
        ("n_odd", ctypes.c_uint64),
        ("hist", ctypes.c_uint64 * 65),
        ("ksum", ctypes.c_uint64),
        ("kmax_seen", ctypes.c_uint32),
        ("n_records", ctypes.c_uint32),
        ("n_exceptions", ctypes.c_uint64),
    ]


class _Record(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("k", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


def build(force: bool = True) -> str:
    """Compile esq_oracle.c into liboracle.so with gcc (plain C, pthreads)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
             "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_prepare.argtypes = [ctypes.c_uint64]
        lib.oracle_prepare.restype = ctypes.c_int
        lib.oracle_nprimes.restype = ctypes.c_size_t
        lib.oracle_is_squarefree.argtypes = [ctypes.c_uint64]
        lib.oracle_is_squarefree.restype = ctypes.c_int
        lib.oracle_mink.argtypes = [ctypes.c_uint64, ctypes.c_uint]
        lib.oracle_mink.restype = ctypes.c_uint
        lib.oracle_verify_range.argtypes = [
            ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint, ctypes.c_int,
            ctypes.c_void_p, ctypes.POINTER(_Summary), ctypes.POINTER(_Record), ctypes.c_size_t,
            ctypes.c_void_p, ctypes.c_size_t]
        lib.oracle_verify_range.restype = ctypes.c_int
        lib.oracle_sieve_bits.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                          ctypes.c_void_p]
        lib.oracle_sieve_bits.restype = ctypes.c_int64
        lib.oracle_mink_many.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint,
                                         ctypes.c_int, ctypes.c_void_p]
        lib.oracle_mink_many.restype = ctypes.c_int
        lib.oracle_sqf_many.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        lib.oracle_sqf_many.restype = ctypes.c_int
        _lib = lib
        return lib


def _threads(nthreads):
    return int(nthreads) if nthreads else (os.cpu_count() or 1)


def _isqrt(x: int) -> int:
    import math
    return math.isqrt(x)


def nprimes(limit: int) -> int:
    """Number of odd primes <= limit in the oracle's own prime list."""
    lib = _load()
    lib.oracle_prepare(int(limit))
    lib.oracle_primes.restype = ctypes.POINTER(ctypes.c_uint32)
    cnt = lib.oracle_nprimes()
    arr = np.ctypeslib.as_array(lib.oracle_primes(), shape=(cnt,))
    return int(np.searchsorted(arr, int(limit), side="right"))


def mink(n: int, kmax: int = 0) -> int:
    """Algorithm 2 for one odd n >= 3: least k >= 1 with n - 2^k >= 1
    squarefree (k <= kmax when kmax > 0); 0 when none is found."""
    lib = _load()
    if lib.oracle_prepare(_isqrt(int(n))) != 0:
        raise MemoryError("oracle prime list")
    return int(lib.oracle_mink(int(n), int(kmax)))


def mink_many(ns, kmax: int = 0, nthreads=None) -> np.ndarray:
    """Algorithm 2 for each odd n of ``ns`` (uint64); returns uint8 least k."""
    lib = _load()
    a = np.ascontiguousarray(np.asarray(ns, dtype=np.uint64))
    out = np.zeros(a.size, dtype=np.uint8)
    if a.size:
        if lib.oracle_mink_many(a.ctypes.data, a.size, int(kmax), _threads(nthreads),
                                out.ctypes.data) != 0:
            raise MemoryError("oracle prime list")
    return out


def is_squarefree_many(ms) -> np.ndarray:
    """Squarefree flag (Section 2: no odd prime square divides m) of odd m >= 1."""
    lib = _load()
    a = np.ascontiguousarray(np.asarray(ms, dtype=np.uint64))
    out = np.zeros(a.size, dtype=np.uint8)
    if a.size:
        if lib.oracle_sqf_many(a.ctypes.data, a.size, out.ctypes.data) != 0:
            raise MemoryError("oracle prime list")
    return out


def sieve_bits(lo: int, hi: int, nthreads=None):
    """Algorithm 1 alone: squarefree flags of the odd m in [lo, hi), m >= 1.

    Returns (m0, n_bits, words) with words a uint64 array, bit i (LSB first)
    set iff m0 + 2i is squarefree; tail bits are 0.
    """
    lib = _load()
    lo = max(int(lo), 1)
    m0 = lo | 1
    n = (int(hi) - m0 + 1) // 2 if hi > m0 else 0
    words = np.zeros((n + 63) // 64, dtype=np.uint64)
    if n:
        got = lib.oracle_sieve_bits(lo, int(hi), _threads(nthreads), words.ctypes.data)
        if got != n:
            raise RuntimeError("oracle_sieve_bits failed")
    return m0, n, words


def verify_range(lo: int, hi: int, kmax: int = 0, per_n: bool = False,
                 nthreads=None, rec_cap: int = 64, exc_cap: int = 1 << 16):
    """Algorithm 2 over every odd n in [lo, hi) with n >= 3 plus the
    aggregates of Section 3 ("Collecting the results"), Table 3 records and
    Table 4 counts.

    Returns a dict: n0, n_odd, hist (65 ints), ksum, kmax_seen, records
    [(n, k)], record_flags (1 for a k = 0 record whose search the limit kmax
    cut short while 2^(kmax+1) < n, else 0), n_records, exceptions [n]
    (ascending, at most exc_cap), n_exceptions, and per_n (uint8 array) when
    requested.
    """
    lib = _load()
    lo, hi = int(lo), int(hi)
    n0 = max(lo, 3) | 1
    n_odd = (hi - n0 + 1) // 2 if hi > n0 else 0
    pern = np.zeros(n_odd, dtype=np.uint8) if per_n else None
    s = _Summary()
    recs = (_Record * max(rec_cap, 1))()
    exc = np.zeros(max(exc_cap, 1), dtype=np.uint64)
    rc = lib.oracle_verify_range(lo, hi, int(kmax), _threads(nthreads),
                                 pern.ctypes.data if pern is not None and n_odd else None,
                                 ctypes.byref(s), recs, rec_cap, exc.ctypes.data, exc_cap)
    if rc != 0:
        raise MemoryError("oracle_verify_range failed")
    nrec = min(s.n_records, rec_cap)
    nexc = min(s.n_exceptions, exc_cap)
    out = {
        "n0": s.n0,
        "n_odd": s.n_odd,
        "hist": [int(x) for x in s.hist],
        "ksum": int(s.ksum),
        "kmax_seen": int(s.kmax_seen),
        "n_records": int(s.n_records),
        "records": [(int(recs[i].n), int(recs[i].k)) for i in range(nrec)],
        "record_flags": [int(recs[i].flags) for i in range(nrec)],
        "n_exceptions": int(s.n_exceptions),
        "exceptions": [int(x) for x in exc[:nexc]],
    }
    if per_n:
        out["per_n"] = pern
    return out
