"""Serving (continuous batching): requests of mixed size and mode arriving
while others run give exactly the result of each interval alone."""
import numpy as np
import pytest
import torch

import oracle
from paper_2411_01964_amd import esq, serve, workloads
from tests.conftest import load_oracle_sample

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def lib_ready():
    esq.init(0, (1 << 50) + (1 << 33))
    for k, v in dict(seg_log2=18, kh=13, block=512, entry_hits=12, tail_cap=1 << 20,
                     medium_max=4095, bucket_cap=0, items_per_wg=4).items():
        esq.set_param(k, v)


KEYS = ("n0", "n_odd", "hist", "ksum", "kmax_seen", "records", "record_flags", "n_records",
        "n_exceptions")


@pytest.mark.parametrize("paced,budget", [(True, 16 << 30), (False, 64 << 20)])
def test_served_results_equal_alone(paced, budget):
    reqs = workloads.poisson_requests(seed=55, rate=4000.0, duration=0.05, log2_len=(8, 22))
    assert len(reqs) > 50
    done, wall, stats = serve.run_stream(reqs, n_streams=3, hbm_budget=budget, warmup_s=0.0,
                                         paced=paced)
    assert stats["requests"] == len(reqs) and stats["batches"] >= 1
    for (t, lo, hi, per_n), r in zip(reqs, done):
        alone = esq.verify_range(lo, hi, per_n=per_n)
        for k in KEYS:
            assert r.result[k] == alone[k], k
        if per_n:
            assert torch.equal(r.result["per_n"], alone["per_n"])


def test_admission_respects_budget():
    srv = serve.Server(n_streams=2, hbm_budget=1 << 20)
    try:
        big = srv.submit(3, 1 << 22, per_n=True)      # alone above the budget: runs by itself
        small = [srv.submit(1001 + 4096 * i, 1001 + 4096 * i + 2000) for i in range(8)]
        assert big.wait(60) is not None
        for r in small:
            assert r.wait(60) is not None
        assert big.result["n_odd"] == (1 << 21) - 1
    finally:
        srv.close()


@pytest.mark.parametrize("paced,budget", [(True, 4 << 30), (False, 1 << 30)])
def test_served_config5_stream_vs_alone_and_oracle(paced, budget):
    """The first 300 requests of the seeded served workload (Poisson arrivals
    at 2000/s, lengths 2^12..2^30 odd n, starts in [3, 2^50), half of them
    per-n), served in the mix -- at their arrival times, or all at once under
    a 1 GiB budget so that admission holds requests back -- equal each
    interval alone, and the oracle: stored aggregates of every request of at
    most 2^13 odd n, the stored least k of 16 seeded n of every other request
    (from the served per-n bytes, or from a per-n call alone for summary
    requests), and the depth of every record-setter recomputed."""
    meta, ns, k, parts = load_oracle_sample("cfg5_sample")
    reqs = workloads.poisson_requests(seed=5, rate=2000.0, duration=11.0)[:300]
    assert len(parts) == len(reqs) == 300
    done, wall, stats = serve.run_stream(reqs, n_streams=3, hbm_budget=budget, warmup_s=0.0,
                                         paced=paced)
    assert stats["requests"] == 300
    full = {(f["lo"], f["hi"]): f for f in meta["full"]}
    rec_n, rec_k = [], []
    for (t, lo, hi, per_n), r, (a, b, start, stop, is_full) in zip(reqs, done, parts):
        assert (a, b) == (lo, hi)
        res = r.result
        alone = esq.verify_range(lo, hi, per_n=True)
        for key in KEYS:
            assert res[key] == alone[key], (key, lo, hi)
        if per_n:
            assert torch.equal(res["per_n"], alone["per_n"]), (lo, hi)
        idx = torch.from_numpy(((ns[start:stop] - np.uint64(res["n0"])) // np.uint64(2))
                               .astype(np.int64)).cuda()
        src = res["per_n"] if per_n else alone["per_n"]
        assert np.array_equal(src[idx].cpu().numpy(), k[start:stop]), (lo, hi)
        if is_full:
            f = full[(lo, hi)]
            assert res["hist"] == f["hist"] and res["ksum"] == f["ksum"], (lo, hi)
            assert res["kmax_seen"] == f["kmax_seen"] and res["n_exceptions"] == f["n_exceptions"]
            assert res["records"] == [tuple(x) for x in f["records"]], (lo, hi)
        rec_n += [n for n, _ in res["records"]]
        rec_k += [kk for _, kk in res["records"]]
        del alone, src
        r.result = None
    assert [int(x) for x in oracle.mink_many(rec_n)] == rec_k
