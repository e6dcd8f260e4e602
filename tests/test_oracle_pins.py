"""Pins of the CPU oracle against facts fixed outside it: brute force over all
divisors, an exact Moebius count, factorisations from sympy, the paper's
worked examples and tables, the Chinese-remainder construction of Section 2's
remark, and the heuristic densities of Table 2.  CPU only."""
import math

import numpy as np
import pytest
import sympy

import oracle
from tests.conftest import read_golden
from paper_2411_01964_amd import workloads


# --------------------------------------------------------------- helpers

def brute_squarefree_odd(limit):
    """sqf[m] for m < limit by striking multiples of d^2 for EVERY d >= 2
    (composite d included) -- not the oracle's prime trial division."""
    sqf = np.ones(limit, dtype=bool)
    d = 2
    while d * d < limit:
        sqf[d * d::d * d] = False
        d += 1
    return sqf


def mobius_upto(n):
    """Moebius function mu(0..n) by a linear sieve (its own code)."""
    mu = np.ones(n + 1, dtype=np.int8)
    mu[0] = 0
    is_comp = np.zeros(n + 1, dtype=bool)
    primes = []
    mu_l = [0] * (n + 1)
    mu_l[1] = 1
    for i in range(2, n + 1):
        if not is_comp[i]:
            primes.append(i)
            mu_l[i] = -1
        for p in primes:
            if i * p > n:
                break
            is_comp[i * p] = True
            if i % p == 0:
                mu_l[i * p] = 0
                break
            mu_l[i * p] = -mu_l[i]
    mu[:] = np.array(mu_l, dtype=np.int8)
    return mu


def q_odd(x, mu):
    """Number of odd squarefree m with 1 <= m <= x:
    sum over odd d with d^2 <= x of mu(d) * #{odd j <= x / d^2}."""
    if x <= 0:
        return 0
    total = 0
    r = math.isqrt(x)
    for d in range(1, r + 1, 2):
        if mu[d]:
            total += int(mu[d]) * ((x // (d * d) + 1) // 2)
    return total


def popcount_words(words):
    return int(sum(bin(int(w)).count("1") for w in words))


def sympy_squarefree(m):
    return all(e == 1 for e in sympy.factorint(m).values())


# ------------------------------------------------- squarefreeness itself

def test_sqf_matches_all_divisor_brute_force():
    limit = 300001
    brute = brute_squarefree_odd(limit)
    m0, n, words = oracle.sieve_bits(1, limit)
    assert m0 == 1 and n == len(range(1, limit, 2))
    bits = np.unpackbits(words.view(np.uint8), bitorder="little")[:n].astype(bool)
    expect = brute[1:limit:2]
    assert np.array_equal(bits, expect)


def test_sqf_matches_sympy_factorisation_large():
    rng = np.random.default_rng(11)
    ms = [int(x) | 1 for x in rng.integers(1 << 30, 1 << 50, size=300, dtype=np.int64)]
    # include known non-squarefree values at scale: p^2 * odd
    ms += [1000003 ** 2 * 7, 9 * 125_899_906_842_597, 33554393 ** 2]
    got = oracle.is_squarefree_many(ms)
    for m, g in zip(ms, got):
        assert bool(g) == sympy_squarefree(m), m


def test_one_is_squarefree_and_prime_squares_are_not():
    got = oracle.is_squarefree_many([1, 9, 25, 49, 121, 169, 2039 ** 2, 3, 15, 105])
    assert list(got) == [1, 0, 0, 0, 0, 0, 0, 1, 1, 1]


@pytest.mark.parametrize("lo,hi", [
    (1, 1 << 20),
    (2, 999_999),
    (1_000_000, 3_000_001),
    ((1 << 40), (1 << 40) + (1 << 16)),
    ((1 << 40) + 7, (1 << 40) + (1 << 16) + 2),
])
def test_sieve_popcount_equals_moebius_count(lo, hi):
    m0, n, words = oracle.sieve_bits(lo, hi)
    mu = mobius_upto(math.isqrt(hi) + 1)
    expect = q_odd(hi - 1, mu) - q_odd(max(lo, 1) - 1, mu)
    assert popcount_words(words) == expect


def test_sieve_bits_conventions():
    # empty ranges
    assert oracle.sieve_bits(10, 10)[1] == 0
    assert oracle.sieve_bits(10, 11)[1] == 0
    # lo even / odd, hi even / odd
    m0, n, w = oracle.sieve_bits(8, 20)      # 9 11 13 15 17 19
    assert (m0, n) == (9, 6)
    assert int(w[0]) == 0b111110             # 9 is not squarefree
    m0, n, w = oracle.sieve_bits(0, 10)      # 1 3 5 7 9
    assert (m0, n) == (1, 5) and int(w[0]) == 0b01111
    m0, n, w = oracle.sieve_bits(25, 26)     # just 25
    assert (m0, n, int(w[0])) == (25, 1, 0)
    # tail bits beyond n are zero
    m0, n, w = oracle.sieve_bits(1, 201)
    assert n == 100 and int(w[1]) >> (100 - 64) == 0


# ---------------------------------------------------- least k (Alg. 2)

def brute_mink(n, kmax=0):
    k = 1
    while (1 << k) < n and (kmax == 0 or k <= kmax):
        m = n - (1 << k)
        d, ok = 2, True
        while d * d <= m:
            if m % (d * d) == 0:
                ok = False
                break
            d += 1
        if ok:
            return k
        k += 1
    return 0


def test_small_n_against_brute_force_including_positivity():
    r = oracle.verify_range(0, 6000, per_n=True)
    assert r["n0"] == 3
    ns = range(3, 6000, 2)
    expect = np.array([brute_mink(n) for n in ns], dtype=np.uint8)
    assert np.array_equal(r["per_n"], expect)
    # n = 3 uses m = 1 (squarefree): k = 1
    assert r["per_n"][0] == 1
    # n = 2^j + 1: n - 2^j = 1 is the last positive candidate
    for j in range(2, 12):
        assert 1 <= oracle.mink((1 << j) + 1) <= j


def test_worked_examples_of_table3_rows_1_to_4():
    # 11: 9 = 3^2 fails, 7 squarefree -> k = 2
    # 29: 27, 25 fail, 21 -> 3;  533: 531, 529, 525 fail, 517 -> 4;
    # 849: 847, 845, 841, 833 fail, 817 -> 5
    assert [oracle.mink(n) for n in (11, 29, 533, 849)] == [2, 3, 4, 5]
    for n, k in ((11, 2), (29, 3), (533, 4), (849, 5)):
        for j in range(1, k):
            assert not sympy_squarefree(n - (1 << j))
        assert sympy_squarefree(n - (1 << k))


def test_every_table3_row_has_depth_m_plus_1():
    rows = read_golden("table3_records.txt")
    ns = [int(n) for _, n in rows]
    got = oracle.mink_many(ns)
    assert [int(g) for g in got] == [int(m) + 1 for m, _ in rows]


def test_table3_records_from_a_full_scan_to_2pow25():
    rows = read_golden("table3_records.txt")
    r = oracle.verify_range(3, 1 << 25)
    expect = [(3, 1)] + [(int(n), int(m) + 1) for m, n in rows if int(n) < (1 << 25)]
    assert r["records"] == expect
    assert sum(r["hist"]) == r["n_odd"] == (1 << 24) - 1
    assert r["ksum"] == sum(k * c for k, c in enumerate(r["hist"]))
    assert r["n_exceptions"] == 0


@pytest.mark.slow
def test_table4_histogram_exactly_below_2pow30():
    rows = read_golden("table4_hist.txt")
    r = oracle.verify_range(3, 1 << 30)
    for k, cnt in rows:
        assert r["hist"][int(k)] == int(cnt), k
    assert sum(r["hist"]) == (1 << 29) - 1
    assert r["ksum"] == 652_756_698
    t3 = [(int(n), int(m) + 1) for m, n in read_golden("table3_records.txt") if int(n) < (1 << 30)]
    assert r["records"] == [(3, 1)] + t3


def test_crt_construction_forces_depth():
    """Remark of Section 2: n = 2^k (mod p_(k+1)^2) for k = 1..l forces the
    least exponent to be at least l + 1, at any magnitude."""
    odd_primes = [3, 5, 7, 11, 13, 17, 19]
    rng = np.random.default_rng(5)
    for ell in range(1, 8):
        mods = [p * p for p in odd_primes[:ell]] + [2]
        res = [(1 << k) % (p * p) for k, p in zip(range(1, ell + 1), odd_primes)] + [1]
        n, M = sympy.ntheory.modular.crt(mods, res)
        n, M = int(n), int(M)
        cands = [n + M * int(t) for t in rng.integers(0, max(1, (1 << 48) // M), size=6)]
        cands = [c for c in cands if c > (1 << (ell + 1))]
        got = oracle.mink_many(cands)
        assert all(int(g) >= ell + 1 for g in got), (ell, cands, got)
        # with the search limited to kmax = ell every such n is an exception
        assert all(int(g) == 0 for g in oracle.mink_many(cands, kmax=ell))


def test_density_against_table2():
    """Least-k frequencies of random odd n near 2^40 against c_l - c_(l-1)
    of Section 2 (recomputed by oracle/constants.py, pinned to Table 2 in
    test_constants.py), binomial sigma (a statistical check, never equality)."""
    from oracle import constants
    p = {l: float(b) for l, _, b in constants.table(m=10**5, lmax=8)}
    ns = workloads.random_odd(seed=21, count=1 << 14, lo=1 << 40, hi=(1 << 40) + (1 << 36))
    got = np.bincount(oracle.mink_many(ns), minlength=21)
    N = len(ns)
    assert got[0] == 0
    for ell in range(1, 7):
        mean = N * p[ell]
        sigma = math.sqrt(N * p[ell] * (1 - p[ell]))
        assert abs(got[ell] - mean) < 6 * sigma + 1, (ell, got[ell], mean)


# ------------------------------------------- records, exceptions, kmax

def records_from_per_n(n0, per_n):
    """Strict prefix maxima of the depth, exceptions (0) counting as
    infinity -- recomputed from the per-n array."""
    out, best = [], 0
    for i, k in enumerate(per_n.tolist()):
        depth = k if k else 1000
        if depth > best:
            out.append((n0 + 2 * i, k))
            best = depth
    return out


@pytest.mark.parametrize("kmax", [1, 2, 3, 4, 6])
def test_kmax_truncation(kmax):
    full = oracle.verify_range(3, 1 << 19, per_n=True)
    cut = oracle.verify_range(3, 1 << 19, kmax=kmax, per_n=True, exc_cap=1 << 20)
    fp = full["per_n"]
    expect_exc = [3 + 2 * int(i) for i in np.nonzero(fp > kmax)[0]]
    assert cut["exceptions"] == expect_exc
    assert cut["n_exceptions"] == cut["hist"][0] == len(expect_exc)
    assert np.array_equal(cut["per_n"], np.where(fp > kmax, 0, fp))
    assert cut["records"] == records_from_per_n(3, cut["per_n"])
    for k in range(1, kmax + 1):
        assert cut["hist"][k] == full["hist"][k]
    # every exception really has no representation with k <= kmax
    for n in expect_exc[:20]:
        for k in range(1, kmax + 1):
            assert not sympy_squarefree(n - (1 << k))


def test_records_semantics_and_threads_are_deterministic():
    lo, hi = (1 << 40) + 12345, (1 << 40) + 12345 + (1 << 14)
    a = oracle.verify_range(lo, hi, per_n=True, nthreads=1)
    b = oracle.verify_range(lo, hi, per_n=True, nthreads=7)
    assert a["hist"] == b["hist"] and a["records"] == b["records"]
    assert np.array_equal(a["per_n"], b["per_n"])
    assert a["records"] == records_from_per_n(a["n0"], a["per_n"])
    assert a["kmax_seen"] == int(a["per_n"].max())
    assert a["n0"] == ((1 << 40) + 12345) | 1


def test_empty_and_degenerate_ranges():
    for lo, hi in ((0, 3), (3, 3), (10, 4), (4, 5), (1, 2)):
        r = oracle.verify_range(lo, hi)
        assert r["n_odd"] == 0 and sum(r["hist"]) == 0 and r["records"] == []
    r = oracle.verify_range(0, 4)
    assert r["n_odd"] == 1 and r["records"] == [(3, 1)]


@pytest.mark.parametrize("kmax", [0, 1, 2, 3])
def test_aggregates_against_brute_force_below_6000(kmax):
    """The oracle's per-k counts, sum of k, maximum k, records (with the
    exception kind) and exceptions over the odd n in [3, 6000), against the
    same aggregates built here from the all-divisor brute force, n by n
    (Section 3, "Collecting the results"; Algorithm 2's report)."""
    r = oracle.verify_range(0, 6000, kmax=kmax, exc_cap=1 << 12)
    hist, ksum, kseen, recs, flags, exc, best = [0] * 65, 0, 0, [], [], [], 0
    for n in range(3, 6000, 2):
        k = brute_mink(n, kmax)
        hist[k] += 1
        ksum += k
        kseen = max(kseen, k)
        depth = k if k else 1000
        if depth > best:
            recs.append((n, k))
            flags.append(1 if k == 0 and kmax and (1 << (kmax + 1)) < n else 0)
            best = depth
        if k == 0:
            exc.append(n)
    assert r["hist"] == hist
    assert r["ksum"] == ksum and r["kmax_seen"] == kseen
    assert r["records"] == recs and r["record_flags"] == flags
    assert r["exceptions"] == exc and r["n_exceptions"] == len(exc)
    if kmax:
        # the first n deeper than kmax is an exception cut short by the limit
        assert recs[-1][1] == 0 and flags[-1] == 1
