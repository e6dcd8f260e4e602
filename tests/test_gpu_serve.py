"""Serving (continuous batching): requests of mixed size and mode arriving
while others run give exactly the result of each interval alone."""
import pytest
import torch

from paper_2411_01964_amd import esq, serve, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def lib_ready():
    esq.init(0, (1 << 50) + (1 << 33))
    for k, v in dict(seg_log2=18, kh=13, block=512, entry_hits=16, tail_cap=1 << 20,
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
