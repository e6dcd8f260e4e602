"""GPU results at the full sizes of the workloads, in the launch configuration
that bench.py times (default knobs, summary mode), checked against what the
paper fixes (Tables 3 and 4), against the oracle on sampled n, and against
properties that hold at any size."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2411_01964_amd import esq, workloads
from tests.conftest import load_oracle_sample, read_golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def lib_ready():
    esq.init(0, (1 << 50) + (1 << 33))
    for k, v in dict(seg_log2=18, kh=13, block=512, entry_hits=12, tail_cap=1 << 20).items():
        esq.set_param(k, v)


def table2():
    """P(least exponent = l), l <= 9, recomputed from Section 2's formulas
    (oracle/constants.py; its digits are pinned to Table 2 on the CPU)."""
    from oracle import constants
    return {l: float(b) for l, _, b in constants.table(m=10**5, lmax=9)}


def check_density(hist, N):
    p = table2()
    for k in range(1, 9):
        pk = p[k]
        mean = N * pk
        sigma = math.sqrt(N * pk * (1 - pk))
        assert abs(hist[k] - mean) <= 6 * sigma + 1, (k, hist[k], mean, sigma)


def check_records_with_oracle(res):
    """Each record-setter's depth recomputed by the oracle; depths increase."""
    ns = [n for n, _ in res["records"]]
    ks = [int(x) for x in oracle.mink_many(ns)]
    assert ks == [k for _, k in res["records"]]
    assert ks == sorted(ks) and len(set(ks)) == len(ks)
    assert res["records"][0][0] == res["n0"]


def test_table4_and_table3_below_2pow30_on_gpu():
    g = esq.verify_range(3, 1 << 30)
    for k, cnt in read_golden("table4_hist.txt"):
        assert g["hist"][int(k)] == int(cnt), k
    assert sum(g["hist"]) == (1 << 29) - 1
    assert g["ksum"] == 652_756_698
    t3 = [(int(n), int(m) + 1) for m, n in read_golden("table3_records.txt") if int(n) < (1 << 30)]
    assert g["records"] == [(3, 1)] + t3
    assert g["kmax_seen"] == 9 and g["n_exceptions"] == 0


@pytest.mark.parametrize("name,samples", [
    ("odd_2pow31_at_2pow40", ("cfg2_random", "cfg2_windows")),
    ("odd_2pow33_below_2pow50", ("cfg3_random", "cfg3_windows"))])
def test_full_interval(name, samples):
    """The benchmarked call over the whole interval, then the same interval in
    per-n mode: equal aggregates, and the per-n bytes equal the oracle's least
    k at 2^20 stored seeded random n and at every n of the stored seeded
    windows (64 of 2^16 n at 2^40, 16 of 2^12 n near 2^50)."""
    lo, hi = workloads.CONFIGS[name]
    g = esq.verify_range(lo, hi)                       # the benchmarked call
    N = g["n_odd"]
    assert N == (hi - (lo | 1) + 1) // 2
    assert sum(g["hist"]) == N and g["status"] == 0 and g["n_exceptions"] == 0
    assert g["ksum"] == sum(k * c for k, c in enumerate(g["hist"]))
    assert g["kmax_seen"] == max(k for k in range(65) if g["hist"][k])
    assert g["kmax_seen"] <= 13                        # Theorem 1
    check_density(g["hist"], N)
    check_records_with_oracle(g)
    # the per-n mode over the same interval: same counts, stored oracle samples
    p = esq.verify_range(lo, hi, per_n=True)
    assert p["hist"] == g["hist"] and p["records"] == g["records"]
    per_n = p["per_n"]
    counts = torch.bincount(per_n, minlength=65).cpu().tolist()
    assert counts[:65] == g["hist"]
    for sname in samples:
        meta, ns, k, parts = load_oracle_sample(sname)
        assert ns.min() >= lo and ns.max() < hi
        idx = torch.from_numpy(((ns - np.uint64(g["n0"])) // np.uint64(2)).astype(np.int64)).cuda()
        got = per_n[idx].cpu().numpy()
        bad = np.nonzero(got != k)[0]
        assert bad.size == 0, (sname, int(bad.size), [(int(ns[i]), int(got[i]), int(k[i])) for i in bad[:5]])
    # record-setters are where the running maximum of per_n increases
    for n, k in g["records"]:
        assert int(per_n[(n - g["n0"]) // 2]) == k
    del per_n, p
    torch.cuda.empty_cache()


@pytest.mark.parametrize("sname", ["cfg2_windows", "cfg3_windows"])
def test_full_interval_windows_vs_oracle(sname):
    """The stored seeded windows inside the benchmarked intervals, each as a
    call of its own: per-n bytes element by element and every aggregate
    (histogram, sum, maximum, records, exceptions) equal the oracle's."""
    meta, ns, k, parts = load_oracle_sample(sname)
    full = {(f["lo"], f["hi"]): f for f in meta["full"]}
    assert len(full) == len(parts) == meta["count"]
    for a, b, start, stop, _ in parts:
        g = esq.verify_range(a, b, per_n=True)
        f = full[(a, b)]
        assert g["hist"] == f["hist"] and g["ksum"] == f["ksum"] and g["kmax_seen"] == f["kmax_seen"]
        assert g["records"] == [tuple(x) for x in f["records"]] and g["n_exceptions"] == f["n_exceptions"]
        assert np.array_equal(g["per_n"].cpu().numpy(), k[start:stop]), (a, b)


def mobius_np(n):
    """mu(0..n): -1 for each prime factor, 0 on a square factor (its own sieve)."""
    mu = np.ones(n + 1, dtype=np.int8)
    mu[0] = 0
    is_p = np.ones(n + 1, dtype=bool)
    is_p[:2] = False
    for p in range(2, math.isqrt(n) + 1):
        if is_p[p]:
            is_p[p * p::p] = False
    for p in np.nonzero(is_p)[0]:
        p = int(p)
        mu[::p] *= -1
        if p * p <= n:
            mu[::p * p] = 0
    return mu


def q_odd_np(x, mu):
    """Odd squarefree m in [1, x]: sum over odd d, d^2 <= x, of
    mu(d) * #{odd multiples of d^2 up to x}."""
    if x <= 0:
        return 0
    d = np.arange(1, math.isqrt(x) + 1, 2, dtype=np.int64)
    return int(np.sum(mu[d].astype(np.int64) * ((x // (d * d) + 1) // 2)))


def popcount_gpu(words):
    """Set bits of an int64 CUDA tensor (SWAR on 32-bit lanes, then bytes)."""
    x = words.view(torch.int32)
    x = x - ((x >> 1) & 0x55555555)
    x = (x & 0x33333333) + ((x >> 2) & 0x33333333)
    x = (x + (x >> 4)) & 0x0F0F0F0F
    return int(x.view(torch.uint8).sum(dtype=torch.int64))


@pytest.mark.parametrize("name", ["odd_2pow31_at_2pow40", "odd_2pow33_below_2pow50"])
def test_sieve_full_interval_moebius_count(name):
    """Algorithm 1 alone over a whole benchmarked interval of odd m: the
    number of set bits equals the exact Moebius count of odd squarefree m in
    it, the bits past the end are clear, and sampled bits match the oracle's
    trial division."""
    lo, hi = workloads.CONFIGS[name]
    m0, n, w = esq.sieve_segment(lo, hi)
    assert m0 == lo | 1 and n == (hi - m0 + 1) // 2
    mu = mobius_np(math.isqrt(hi) + 1)
    assert popcount_gpu(w) == q_odd_np(hi - 1, mu) - q_odd_np(lo - 1, mu)
    if n % 64:
        assert int(w[-1]) >> (n % 64) == 0
    i = workloads.random_odd(seed=11, count=512, lo=0, hi=2 * n).astype(np.int64) // 2
    bits = ((w[torch.from_numpy(i // 64).cuda()] >> torch.from_numpy(i % 64).cuda()) & 1).cpu().numpy()
    ms = (np.uint64(m0) + 2 * i.astype(np.uint64))
    assert np.array_equal(bits.astype(np.uint8), oracle.is_squarefree_many(ms))
    del w
    torch.cuda.empty_cache()
