"""esq_verify_range_noalloc, the entry point for callers that cannot allocate
device memory, called through the C-ABI with raw device pointers: its
results equal esq_verify_range's bit for bit, call after call on the shared
static scratch (a smaller input after a larger one included), and an
interval whose scratch exceeds the static array is refused before anything
is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2411_01964_amd import esq, workloads

pytestmark = pytest.mark.gpu

KEYS = ("n0", "n_odd", "hist", "ksum", "kmax_seen", "records", "record_flags", "n_records",
        "n_exceptions", "exceptions", "status")
DEFAULTS = dict(seg_log2=18, kh=13, block=512, entry_hits=12, tail_cap=1 << 20,
                medium_max=4095, bucket_cap=0)


@pytest.fixture(scope="module", autouse=True)
def lib_ready():
    esq.init(0, (1 << 50) + (1 << 33))
    for k, v in DEFAULTS.items():
        esq.set_param(k, v)
    yield
    for k, v in DEFAULTS.items():
        esq.set_param(k, v)


def noalloc_call(lo, hi, kmax=0, per_n=False, exceptions_cap=0):
    """One esq_verify_range_noalloc call with caller-made outputs; returns the
    parsed result (per-n bytes as a CUDA tensor)."""
    n0 = max(lo, 3) | 1
    n_odd = (hi - n0 + 1) // 2 if hi > n0 else 0
    dev = torch.device("cuda", 0)
    summary = torch.full((esq.SUMMARY_BYTES,), 0xA5, dtype=torch.uint8, device=dev)
    records = torch.full((esq.ESQ_RECORDS_CAP * esq.RECORD_BYTES,), 0xA5, dtype=torch.uint8,
                         device=dev)
    exc = torch.zeros(max(exceptions_cap, 1), dtype=torch.int64, device=dev)
    mink = torch.full((max(n_odd, 1),), 0xEE, dtype=torch.uint8, device=dev) if per_n else None
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    rc = esq.lib().esq_verify_range_noalloc(
        lo, hi, kmax, ctypes.c_void_p(mink.data_ptr()) if per_n else None,
        ctypes.c_void_p(summary.data_ptr()), ctypes.c_void_p(records.data_ptr()),
        ctypes.c_void_p(exc.data_ptr()) if exceptions_cap else None, exceptions_cap,
        ctypes.c_void_p(stream.cuda_stream))
    assert rc == 0, esq.lib().esq_last_error()
    torch.cuda.synchronize()
    out = esq._parse(summary.cpu().numpy().tobytes(), records.cpu().numpy().tobytes())
    nexc = min(out["n_exceptions"], exceptions_cap)
    out["exceptions"] = [int(x) for x in exc[:nexc].cpu().tolist()] if nexc else []
    if per_n:
        out["per_n"] = mink[:n_odd]
    return out


def check_same(got, want, per_n):
    for k in KEYS:
        assert got[k] == want[k], k
    if per_n:
        assert torch.equal(got["per_n"], want["per_n"])


CASES = [
    # (lo, hi, kmax, per_n, exceptions_cap): a larger call, then a smaller one
    ((1 << 40) + 1, (1 << 40) + (1 << 25), 0, True, 0),
    (3, (1 << 20) + 1, 0, True, 0),
    (3, (1 << 22) + 1, 3, False, 4096),
    (1001, 1001 + 2 * 3000, 2, True, 64),
    ((1 << 50) - (1 << 22) + 1, (1 << 50), 0, False, 0),
    (5, 5, 0, True, 0),
]


def test_noalloc_equals_verify_range_call_after_call():
    for lo, hi, kmax, per_n, cap in CASES:
        want = esq.verify_range(lo, hi, kmax=kmax, per_n=per_n, exceptions_cap=cap, check=False)
        got = noalloc_call(lo, hi, kmax, per_n, cap)
        check_same(got, want, per_n)


def test_noalloc_workload_interval_then_smaller():
    """The benchmarked interval (2^33 odd n just below 2^50) fits the static
    scratch; a much smaller interval right after it on the same scratch."""
    lo, hi = workloads.CONFIGS["odd_2pow33_below_2pow50"]
    need = esq.scratch_bytes([lo], [hi])
    assert need <= esq.ESQ_NOALLOC_SCRATCH_MAX
    want = esq.verify_range(lo, hi)
    got = noalloc_call(lo, hi)
    check_same(got, {**want, "exceptions": []}, False)
    a, b = lo + (1 << 30), lo + (1 << 30) + (1 << 16)
    want = esq.verify_range(a, b, per_n=True)
    got = noalloc_call(a, b, per_n=True)
    check_same(got, {**want, "exceptions": []}, True)


def test_noalloc_allocates_no_device_memory():
    lo, hi = (1 << 45) + 1, (1 << 45) + (1 << 24)
    noalloc_call(lo, hi, per_n=True)           # outputs of this shape already cached by torch
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(0)[0]
    for _ in range(3):
        noalloc_call(lo, hi, per_n=True)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info(0)[0] == free0


def test_noalloc_refuses_scratch_above_the_static_array():
    lo, hi = (1 << 50) - (1 << 38) + 1, 1 << 50
    assert esq.scratch_bytes([lo], [hi]) > esq.ESQ_NOALLOC_SCRATCH_MAX
    summary = torch.zeros(esq.SUMMARY_BYTES, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    rc = esq.lib().esq_verify_range_noalloc(lo, hi, 0, None, ctypes.c_void_p(summary.data_ptr()),
                                            None, None, 0, None)
    assert rc == -2                            # ESQ_ERANGE
    assert b"ESQ_NOALLOC_SCRATCH_MAX" in esq.lib().esq_last_error()
    torch.cuda.synchronize()
    assert int(summary.sum()) == 0             # nothing was enqueued
    # and the next call on the scratch is unaffected
    want = esq.verify_range(3, 1 << 18, per_n=True)
    got = noalloc_call(3, 1 << 18, per_n=True)
    check_same(got, {**want, "exceptions": []}, True)


def test_noalloc_argument_errors():
    L = esq.lib()
    assert L.esq_verify_range_noalloc(3, 100, 0, None, None, None, None, 0, None) == -1
    s = torch.zeros(esq.SUMMARY_BYTES, dtype=torch.uint8, device="cuda")
    p = ctypes.c_void_p(s.data_ptr())
    assert L.esq_verify_range_noalloc(100, 3, 0, None, p, None, None, 0, None) == -1
    assert L.esq_verify_range_noalloc(3, 100, 64, None, p, None, None, 0, None) == -1
    assert L.esq_verify_range_noalloc(3, 100, 0, None, p, None, None, 4, None) == -1
    assert L.esq_verify_range_noalloc(3, 1 << 55, 0, None, p, None, None, 0, None) == -2
    assert np.all(s.cpu().numpy() == 0)
