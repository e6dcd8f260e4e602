"""Pins of the heuristic-constants engine (oracle/constants.py) against what
Section 2 prints and against the mathematics it rests on."""
import itertools
import math

import mpmath
import pytest

from oracle import constants as C
from tests.conftest import read_golden

M_FAST = 10**5   # Lemma 2 cut-off for the tests: |1 - f| < 4e-25


def same_digits(value, text):
    """value agrees with a printed decimal in every printed digit: the tables
    print 'x.xxxx...', truncated or rounded, so |value - printed| < one unit
    of the last printed digit."""
    mant, ex = (text.split("e") + ["0"])[:2]
    frac = mant.split(".")[1] if "." in mant else ""
    unit = mpmath.mpf(10) ** (int(ex) - len(frac))
    return abs(mpmath.mpf(value) - mpmath.mpf(text)) < unit


def test_zeta_closed_forms():
    """d'_1 = 9/pi^2 and d_1 = 8/pi^2 (prod over all primes of 1 - p^-2 is
    1/zeta(2) = 6/pi^2, with the factors of 2 and 3 removed)."""
    with mpmath.workdps(40):
        assert abs(C.d_prime(1, M_FAST) - 9 / mpmath.pi ** 2) < mpmath.mpf(10) ** -38
        assert abs(C.d(1, M_FAST) - 8 / mpmath.pi ** 2) < mpmath.mpf(10) ** -38


@pytest.mark.parametrize("k", [2, 3, 7, 13, 20])
def test_lemma2_against_plain_product(k):
    """d'_k from Lemma 2 against the plain truncated product over
    5 <= p <= 2*10^5: the two differ only by the factor of the primes above
    the cut, prod (1 - k/p^2) ~ exp(-k * sum_{p > M} p^-2), which lies in
    (1 - 2k/(M ln M), 1)."""
    M = 2 * 10**5
    with mpmath.workdps(40):
        plain = mpmath.mpf(1)
        for p in C._primes_upto(M):
            if p >= 5:
                plain *= 1 - mpmath.mpf(k) / (p * p)
        ratio = C.d_prime(k, M_FAST) / plain
        assert 1 - 2 * k / (M * math.log(M)) < ratio < 1, (k, ratio)


def test_lemma1_error_term():
    """Lemma 1 states |e(x)| < 18 x^3 for e(x) = log(1 - kx) - k log(1 - x) -
    binom(k, 2) log(1 - x^2).  The x^3 coefficient of e is -(k^3 - k)/3, so the
    stated bound fails once (k^3 - k)/3 > 18 (k >= 5); the reading used here
    is |e(x)| <= (k^3 - k)/3 x^3 (1 + O(kx)).  Lemma 2's tail factor then obeys
    |log f| <~ (k^3 - k)/15 m^-5, still far below the printed digits at
    m = 10^7."""
    with mpmath.workdps(50):
        for k in (2, 5, 11, 20):
            x = mpmath.mpf(1) / 10**8
            e = mpmath.log(1 - k * x) - k * mpmath.log(1 - x) - math.comb(k, 2) * mpmath.log(1 - x * x)
            coeff = e / x**3
            assert abs(coeff + mpmath.mpf(k**3 - k) / 3) < 1e-5 * k**4, (k, coeff)
        k, x = 20, mpmath.mpf(1) / 49  # p = 7, within Lemma 2's range p > m > 5
        e = mpmath.log(1 - k * x) - k * mpmath.log(1 - x) - math.comb(k, 2) * mpmath.log(1 - x * x)
        assert abs(e) > 18 * x**3


def test_lemma2_cutoff_invariance():
    """Two cut-offs m = 10^4 and 10^5 agree within the tail bound
    (k^3 - k)/15 m^-5 (the corrected Lemma 1 term)."""
    with mpmath.workdps(45):
        for k in (2, 5, 11, 20):
            a, b = C.d_prime(k, 10**4), C.d_prime(k, M_FAST)
            bound = (k**3 - k) / 15 * 1e-20 + 1e-30
            assert abs(a / b - 1) < bound, (k, a / b - 1, bound)


@pytest.mark.parametrize("l", [1, 5, 8, 12])
def test_subset_counts_brute_force(l):
    """The residue-class count behind equation (cell>6) against all 2^l subsets."""
    N = C._subset_counts(l)
    brute = [[0] * 7 for _ in range(l + 1)]
    for r in range(l + 1):
        for I in itertools.combinations(range(1, l + 1), r):
            brute[len(I)][len({k % 6 for k in I})] += 1
    assert N == brute
    assert sum(map(sum, N)) == 2 ** l


@pytest.mark.parametrize("l", range(1, 7))
def test_two_formulas_agree_for_small_l(l):
    """For l <= 6 the binomial form over d_m and equation (cell>6) over d'_m
    are the same number (|I mod 6| = |I| there)."""
    with mpmath.workdps(45):
        assert abs(C.c_small(l, M_FAST) - C.c(l, M_FAST)) < mpmath.mpf(10) ** -40


def test_table1():
    """Table 1 (d_l, c_l, 1 - c_l for l <= 6), every printed digit."""
    for row in read_golden("table1_dl_cl.txt"):
        l = int(row[0])
        assert same_digits(C.d(l, M_FAST), row[1]), ("d", row)
        assert same_digits(C.c_small(l, M_FAST), row[2]), ("c", row)
        assert same_digits(1 - C.c_small(l, M_FAST), row[3]), ("1-c", row)


def test_table2():
    """Table 2 (1 - c_l and c_l - c_(l-1), l <= 20), every printed digit.
    One printed entry, 1 - c_13 = 1.5662e-16, disagrees with the table's own
    neighbours: (1 - c_12) - (c_13 - c_12) = 8.7820e-16 - 7.2190e-16 =
    1.5630e-16.  That entry is checked against its neighbours instead."""
    rows = {int(r[0]): r for r in read_golden("table2_probabilities.txt")}
    computed = {l: (a, b) for l, a, b in C.table(m=10**6)}
    for l, row in rows.items():
        a, b = computed[l]
        assert same_digits(b, row[2]), ("c_l - c_l-1", row, b)
        if l == 13:
            implied = float(rows[12][1]) - float(row[2])
            assert abs(float(a) - implied) < 1e-20
            continue
        assert same_digits(a, row[1]), ("1 - c_l", row, a)


def test_moments():
    """The section's expected least exponent 1.215854247598..., E_S =
    0.607927123799... S, single-instance sigma 0.476... and sigma_S =
    0.336... sqrt(S)."""
    mo = C.moments(m=M_FAST)
    assert same_digits(mo["mean"], "1.215854247598")
    assert same_digits(mo["E_S_coeff"], "0.607927123799")
    assert same_digits(mo["sd"], "0.476")
    assert same_digits(mo["sigma_S_coeff"], "0.336")


def test_table4_counts_near_heuristic():
    """Table 4's exact counts over the odd n < 2^30 against N (c_l - c_(l-1)),
    N = 2^29, within 6 binomial sigma (a statistical statement)."""
    p = {l: float(b) for l, a, b in C.table(m=M_FAST, lmax=9)}
    N = 1 << 29
    for k, cnt in read_golden("table4_hist.txt"):
        k, cnt = int(k), int(cnt)
        if 1 <= k <= 9:
            sigma = math.sqrt(N * p[k] * (1 - p[k]))
            assert abs(cnt - N * p[k]) < 6 * sigma + 1, (k, cnt, N * p[k])
