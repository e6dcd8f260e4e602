"""Long scans on the GPU against the paper's printed results: Table 3's
record-setters (smallest odd n needing k = m + 1) with their minimality,
Table 4's counts, and the whole run below 2^50 (k_sum and Theorem 1)."""
import os

import pytest

from paper_2411_01964_amd import esq, scan
from tests.conftest import read_golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def lib_ready():
    esq.init(0, (1 << 50) + (1 << 33))
    for k, v in dict(seg_log2=18, kh=13, block=512, entry_hits=12, tail_cap=1 << 20,
                     medium_max=4095, bucket_cap=0, items_per_wg=4).items():
        esq.set_param(k, v)


def table3(limit):
    return [(3, 1)] + [(int(n), int(m) + 1) for m, n in read_golden("table3_records.txt")
                       if int(n) < limit]


def test_scan_below_2pow42_gives_table3_rows_up_to_m10():
    r = scan.scan(3, 1 << 42, chunk=1 << 38)
    assert r["records"] == table3(1 << 42)
    assert r["kmax_seen"] == 11 and r["n_exceptions"] == 0 and r["status"] == 0
    assert sum(r["hist"]) == r["n_odd"] == (1 << 41) - 1
    # the first 2^30 integers inside the chunked scan: Table 4 again
    s = scan.scan(3, 1 << 30, chunk=1 << 27)
    for k, cnt in read_golden("table4_hist.txt"):
        assert s["hist"][int(k)] == int(cnt)


def test_full_run_below_2pow50():
    """Section 4: all odd 1 < n < 2^50 -- k_sum, Theorem 1 (k <= 13), and
    every Table 3 row with its minimality."""
    golden = {r[0]: int(r[1]) for r in read_golden("ksum_2pow50.txt")}
    r = scan.scan(3, 1 << 50, chunk=1 << 42)
    assert r["ksum"] == golden["ksum"]
    assert r["kmax_seen"] == golden["max_k"]
    assert r["records"] == table3(1 << 50)
    assert r["n_exceptions"] == 0 and r["status"] == 0
    assert sum(r["hist"]) == r["n_odd"] == (1 << 49) - 1
