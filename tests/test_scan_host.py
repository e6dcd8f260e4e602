"""Host logic of the long-scan driver (chunking, exact merging, checkpoint
and resume, retry), run on the CPU with the oracle standing in for the GPU
call.  The merged aggregates must equal the oracle over the whole range."""
import json

import pytest

import oracle
from paper_2411_01964_amd import scan


class Done:
    def __init__(self, r):
        self.r = r

    def result(self):
        return self.r


def oracle_async(kmax=0, fail_at=None, calls=None):
    calls = calls if calls is not None else []

    def start(lo, hi):
        calls.append((lo, hi))
        if fail_at is not None and len(calls) == fail_at:
            class Boom:
                def result(self):
                    raise RuntimeError("injected launch failure")
            return Boom()
        return Done(oracle.verify_range(lo, hi, kmax=kmax, exc_cap=1 << 16))
    return start


KEYS = ("n0", "n_odd", "hist", "ksum", "kmax_seen", "records", "n_exceptions", "exceptions")


@pytest.mark.parametrize("lo,hi,chunk,kmax", [
    (3, 1 << 16, 1000, 0), (0, 5000, 7, 0), (10, 20000, 4096, 2), (1 << 30, (1 << 30) + 9999, 777, 0),
])
def test_chunked_scan_equals_one_call(lo, hi, chunk, kmax):
    whole = oracle.verify_range(lo, hi, kmax=kmax, exc_cap=1 << 16)
    got = scan.scan(lo, hi, chunk=chunk, verify_async=oracle_async(kmax))
    for k in KEYS:
        assert got[k] == whole[k], k


def test_resume_after_interruption_and_damaged_tail(tmp_path):
    ck = str(tmp_path / "scan.jsonl")
    lo, hi, chunk = 3, 40000, 3000
    whole = oracle.verify_range(lo, hi)
    # first run stops after a few chunks (the range simply ends early)
    scan.scan(lo, lo + 4 * chunk, chunk=chunk, checkpoint=ck, verify_async=oracle_async())
    lines = open(ck).read().splitlines()
    assert len(lines) == 4
    # damage: a truncated last line and a checksum mismatch are recomputed
    with open(ck, "w") as f:
        f.write("\n".join(lines[:2]) + "\n")
        bad = json.loads(lines[2])
        bad["summary"]["ksum"] += 1
        f.write(json.dumps(bad) + "\n")
        f.write(lines[3][: len(lines[3]) // 2])
    calls = []
    got = scan.scan(lo, hi, chunk=chunk, checkpoint=ck, verify_async=oracle_async(calls=calls))
    for k in KEYS:
        assert got[k] == whole[k], k
    assert calls[0] == (lo + 2 * chunk, lo + 3 * chunk)   # resumed after the 2 intact chunks
    again = []
    got2 = scan.scan(lo, hi, chunk=chunk, checkpoint=ck, verify_async=oracle_async(calls=again))
    assert again == [] and got2 == got


def test_failed_chunk_is_retried():
    lo, hi = 3, 30000
    whole = oracle.verify_range(lo, hi)
    got = scan.scan(lo, hi, chunk=2500, verify_async=oracle_async(fail_at=3))
    for k in KEYS:
        assert got[k] == whole[k], k


def test_record_merge_with_exceptions_counts_them_deepest():
    a = {"n0": 3, "n_odd": 2, "hist": [0] * 65, "ksum": 0, "kmax_seen": 2,
         "records": [(3, 1), (11, 2)], "n_exceptions": 0, "exceptions": [], "status": 0}
    b = {"n0": 13, "n_odd": 2, "hist": [0] * 65, "ksum": 0, "kmax_seen": 3,
         "records": [(13, 1), (29, 0)], "n_exceptions": 1, "exceptions": [29], "status": 0}
    c = {"n0": 31, "n_odd": 1, "hist": [0] * 65, "ksum": 0, "kmax_seen": 9,
         "records": [(31, 9)], "n_exceptions": 0, "exceptions": [], "status": 0}
    m = scan.merge(scan.merge(a, b), c)
    assert m["records"] == [(3, 1), (11, 2), (29, 0)]
    assert m["exceptions"] == [29] and m["kmax_seen"] == 9


def test_resume_with_another_chunk_size_and_a_larger_end(tmp_path):
    """A scan resumed with a different chunk size and a larger hi continues
    from the end of the intact checkpoint: nothing skipped, nothing twice."""
    ck = str(tmp_path / "scan.jsonl")
    lo = 3
    scan.scan(lo, lo + 9000, chunk=3000, checkpoint=ck, verify_async=oracle_async())
    calls = []
    got = scan.scan(lo, 40000, chunk=6000, checkpoint=ck, verify_async=oracle_async(calls=calls))
    whole = oracle.verify_range(lo, 40000)
    for k in KEYS:
        assert got[k] == whole[k], k
    assert got["n_odd"] == 19999
    assert calls[0] == (lo + 9000, lo + 9000 + 6000)


def test_checkpoint_of_another_scan_is_rejected(tmp_path):
    ck = str(tmp_path / "scan.jsonl")
    scan.scan(3, 9003, chunk=3000, checkpoint=ck, verify_async=oracle_async())
    with pytest.raises(ValueError, match="another scan"):
        scan.scan(3, 20000, chunk=3000, checkpoint=ck, kmax=2, verify_async=oracle_async(kmax=2))
    with pytest.raises(ValueError, match="another scan"):
        scan.scan(5, 20000, chunk=3000, checkpoint=ck, verify_async=oracle_async())
    with pytest.raises(ValueError, match="past the end"):
        scan.scan(3, 5000, chunk=3000, checkpoint=ck, verify_async=oracle_async())
