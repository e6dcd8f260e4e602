"""The batched form (many intervals in one persistent launch with a device work
queue) gives, per interval, exactly what the interval gives alone, and what
the oracle gives."""
import numpy as np
import pytest
import torch

import oracle
from paper_2411_01964_amd import esq, workloads
from tests.conftest import load_oracle_sample

pytestmark = pytest.mark.gpu
DEFAULTS = dict(seg_log2=18, kh=13, block=512, entry_hits=12, tail_cap=1 << 20,
                medium_max=4095, bucket_cap=0, items_per_wg=4, cof_weight=60)


@pytest.fixture(scope="module", autouse=True)
def lib_ready():
    esq.init(0, (1 << 50) + (1 << 33))
    for k, v in DEFAULTS.items():
        esq.set_param(k, v)
    yield
    for k, v in DEFAULTS.items():
        esq.set_param(k, v)


KEYS = ("n0", "n_odd", "hist", "ksum", "kmax_seen", "records", "record_flags", "n_records",
        "n_exceptions")


def same(a, b):
    for k in KEYS:
        assert a[k] == b[k], k


def mixed_intervals(seed, count, log2_len=(4, 17)):
    lo, hi = workloads.batch_intervals(seed=seed, count=count, log2_len=log2_len,
                                       start_range=(3, 1 << 50))
    # edge cases: empty, tiny, near zero, even bounds, overlapping another entry
    lo += [3, 0, 10, 1 << 40, 1 << 20, lo[0]]
    hi += [3, 4, 11, (1 << 40) + 2, (1 << 20) + 1000, hi[0]]
    return lo, hi


@pytest.mark.parametrize("kw", [dict(), dict(seg_log2=12, items_per_wg=1), dict(kh=4),
                                 dict(bucket_cap=1, medium_max=101), dict(cof_weight=1),
                                 dict(cof_weight=10000)])
def test_batch_equals_alone(kw):
    for k, v in DEFAULTS.items():
        esq.set_param(k, kw.get(k, v))
    lo, hi = mixed_intervals(41, 40)
    per_n = [i % 3 == 0 for i in range(len(lo))]
    batch = esq.verify_batch(lo, hi, per_n=per_n)
    assert len(batch) == len(lo)
    for i, (a, b) in enumerate(zip(lo, hi)):
        alone = esq.verify_range(a, b, per_n=per_n[i])
        same(batch[i], alone)
        if per_n[i]:
            assert torch.equal(batch[i]["per_n"], alone["per_n"]), i


def test_batch_vs_oracle():
    for k, v in DEFAULTS.items():
        esq.set_param(k, v)
    lo, hi = workloads.batch_intervals(seed=43, count=12, log2_len=(6, 12),
                                       start_range=(1 << 30, 1 << 44))
    batch = esq.verify_batch(lo, hi, per_n=[True] * len(lo))
    for i, (a, b) in enumerate(zip(lo, hi)):
        o = oracle.verify_range(a, b, per_n=True)
        same(batch[i], o)
        assert np.array_equal(batch[i]["per_n"].cpu().numpy(), o["per_n"]), i


def test_batch_kmax_and_repeat():
    for k, v in DEFAULTS.items():
        esq.set_param(k, v)
    lo, hi = mixed_intervals(44, 20, log2_len=(8, 14))
    a = esq.verify_batch(lo, hi, kmax=2)
    b = esq.verify_batch(lo, hi, kmax=2)
    for i, (x, y) in enumerate(zip(lo, hi)):
        same(a[i], b[i])
        same(a[i], esq.verify_range(x, y, kmax=2))


def test_batch_workload_equals_alone_and_oracle():
    """The seeded batched workload in full: 4096 intervals (lengths
    2^16..2^28 odd n, starts in [2^30, 2^50)) in one launch, as benchmarked,
    equal each interval alone for all 4096; then the same batch in per-n
    mode, in chunks of intervals, gives the same aggregates and the oracle's
    least k at 64 stored seeded n of every interval."""
    for k, v in DEFAULTS.items():
        esq.set_param(k, v)
    lo, hi = workloads.batch_intervals(seed=4, count=4096)
    batch = esq.verify_batch(lo, hi)
    pend = [esq.verify_range_async(a, b) for a, b in zip(lo, hi)]
    for i, p in enumerate(pend):
        same(batch[i], p.result())
    del pend
    meta, ns, k, parts = load_oracle_sample("cfg4_sample")
    assert len(parts) == 4096
    budget = 1 << 32                          # per-n bytes per chunk
    i = 0
    while i < 4096:
        j, total = i, 0
        while j < 4096 and (j == i or total + batch[j]["n_odd"] <= budget):
            total += batch[j]["n_odd"]
            j += 1
        res = esq.verify_batch(lo[i:j], hi[i:j], per_n=[True] * (j - i))
        for t in range(i, j):
            a, b, start, stop, _ = parts[t]
            assert (a, b) == (lo[t], hi[t])
            r = res[t - i]
            same(r, batch[t])
            idx = torch.from_numpy(((ns[start:stop] - np.uint64(r["n0"])) // np.uint64(2))
                                   .astype(np.int64)).cuda()
            got = r["per_n"][idx].cpu().numpy()
            assert np.array_equal(got, k[start:stop]), (t, a, b)
        del res
        torch.cuda.empty_cache()
        i = j


def test_prepared_batch_and_graph_replays():
    """A prepared batch launched plainly and as a replayed hipGraph, with
    eager work and synchronisations between replays: every replay equals the
    eager result."""
    for k, v in DEFAULTS.items():
        esq.set_param(k, v)
    lo, hi = mixed_intervals(45, 24, log2_len=(8, 16))
    eager = esq.verify_batch(lo, hi)
    pb = esq.PreparedBatch(lo, hi)
    try:
        pb.launch(graph=False)
        for i, r in enumerate(pb.results()):
            same(r, eager[i])
        side = torch.cuda.Stream()
        for rep in range(3):
            pb.launch(graph=True, stream=side if rep % 2 else None)
            torch.cuda.synchronize()
            x = esq.verify_range(lo[rep], hi[rep])       # eager work in between
            same(x, eager[rep])
            for i, r in enumerate(pb.results()):
                same(r, eager[i])
    finally:
        pb.close()


def test_stale_prepared_batch_is_refused():
    """A prepared batch holds the library's resident tables: after esq_init
    replaces them (a larger max_hi) its launch is refused before anything is
    enqueued, and a batch prepared afterwards runs."""
    for k, v in DEFAULTS.items():
        esq.set_param(k, v)
    lo, hi = mixed_intervals(46, 8, log2_len=(8, 12))
    eager = esq.verify_batch(lo, hi)
    pb = esq.PreparedBatch(lo, hi)
    try:
        pb.launch(graph=True)
        for i, r in enumerate(pb.results()):
            same(r, eager[i])
        esq.init(0, (1 << 52) + 1)             # extends the prime table
        with pytest.raises(esq.EsqError) as ei:
            pb.launch(graph=True)
        assert ei.value.code == -1 and "stale" in str(ei.value)
    finally:
        pb.close()
    pb = esq.PreparedBatch(lo, hi)
    try:
        pb.launch(graph=True)
        for i, r in enumerate(pb.results()):
            same(r, eager[i])
    finally:
        pb.close()


def test_scratch_bytes_reports_the_plan():
    """esq_scratch_bytes: the library's scratch for a batch grows with the
    segments it covers and with a listed tail; empty batches take none."""
    for k, v in DEFAULTS.items():
        esq.set_param(k, v)
    assert esq.scratch_bytes([], []) == 0
    small = esq.scratch_bytes([(1 << 40) + 1], [(1 << 40) + (1 << 20)])
    large = esq.scratch_bytes([(1 << 40) + 1], [(1 << 40) + (1 << 34)])
    assert 0 < small < large
    lo, hi = workloads.batch_intervals(seed=4, count=64)
    assert esq.scratch_bytes(lo, hi) >= max(esq.scratch_bytes([a], [b]) for a, b in zip(lo, hi)) // 2
    # kmax at or below the in-LDS depth: no tail list
    assert esq.scratch_bytes([(1 << 40) + 1], [(1 << 40) + (1 << 30)], kmax=3) < \
        esq.scratch_bytes([(1 << 40) + 1], [(1 << 40) + (1 << 30)])
