"""Heuristic constants of Section 2 ("Heuristic arguments"), recomputed.

TEST INFRASTRUCTURE ONLY: the density checks in tests/ compare measured
least-k histograms with these a-priori probabilities.  Nothing on the HIP
path imports this module.

Definitions (Section 2):
  * A_k: n - 2^k is squarefree, for a random odd n.
  * c_l = P(A_1 or ... or A_l); c_l - c_(l-1) = P(least exponent is l), c_0 = 0.
  * d_m = prod over odd primes p of (1 - m/p^2); d'_m = the same over p >= 5.

Under the independence assumption of the section, inclusion-exclusion gives
equation (cellPIE).  For l <= 6 the residues 2^k (k in I) are distinct modulo
every p^2, which collapses it to a binomial sum over d_m.  For 7 <= l <= 20
only p = 3 identifies exponents (2^6 = 1 mod 9; the first identification for
p >= 5 is 2^20 = 1 mod 25), which is equation (cell>6):
  c_l = sum over nonempty I of (-1)^(|I|-1) (1 - |I mod 6|/9) d'_|I|.
d'_k comes from Lemma 2 (the "dkprime" lemma): the zeta-function values
prod_{p>=5}(1 - p^-2) = 9/pi^2 and prod_{p>=5}(1 - p^-4) = 486/(5 pi^4)
carry the tail p > m, the primes 5 <= p <= m are multiplied out, and the
remaining factor f is close to 1.  (The lemma states |1 - f| < 4 m^-5 from
Lemma 1's |e(x)| < 18 x^3; the x^3 coefficient of that error is really
-(k^3 - k)/3, so the tail is about (k^3 - k)/15 m^-5 -- below 10^-30 at
m = 10^7, too small to move any printed digit.)

The finite products are exact-to-rounding fixed-point integers (2^-Q per
factor), the rest is mpmath at `dps` digits.
"""
from __future__ import annotations

import math
from functools import lru_cache

import mpmath
import numpy as np

Q = 256  # fixed-point fraction bits of the finite prime products


def _primes_upto(m: int) -> list:
    """Odd primes 3 <= p <= m (sieve of Eratosthenes)."""
    if m < 3:
        return []
    s = np.ones(m + 1, dtype=bool)
    s[:2] = False
    s[4::2] = False
    for p in range(3, math.isqrt(m) + 1, 2):
        if s[p]:
            s[p * p::2 * p] = False
    return [int(p) for p in np.nonzero(s)[0] if p >= 3]


@lru_cache(maxsize=8)
def _finite_products(m: int, kmax: int = 20):
    """Fixed-point (scale 2^Q) values over the primes 5 <= p <= m of
    prod (1 - k/p^2) for k = 1..kmax, P2 = prod (1 - p^-2)^-1 and
    P4 = prod (1 - p^-4)^-1 (the last two as reciprocals: prod (1 - p^-a))."""
    one = 1 << Q
    acc = [one] * (kmax + 1)
    a4 = one
    for p in _primes_upto(m):
        if p < 5:
            continue
        q = p * p
        for k in range(1, kmax + 1):
            acc[k] = acc[k] * (q - k) // q
        q2 = q * q
        a4 = a4 * (q2 - 1) // q2
    return acc, a4  # acc[1] = prod (1 - p^-2) = 1 / P2; a4 = 1 / P4


def d_prime(k: int, m: int = 10**7, dps: int = 45):
    """d'_k = prod_{p>=5} (1 - k/p^2) by Lemma 2 with cut-off m (mpf).
    Relative error about (k^3 - k)/15 m^-5 plus the fixed-point rounding."""
    if not 1 <= k <= 20:
        raise ValueError("k must be in 1..20")
    with mpmath.workdps(dps):
        if k == 1:
            return 9 / mpmath.pi ** 2
        acc, a4 = _finite_products(m)
        scale = mpmath.mpf(2) ** Q
        fin_k = mpmath.mpf(acc[k]) / scale      # prod_{5<=p<=m} (1 - k/p^2)
        inv_p2 = mpmath.mpf(acc[1]) / scale     # 1 / P_{2,m}
        inv_p4 = mpmath.mpf(a4) / scale         # 1 / P_{4,m}
        b = k * (k - 1) // 2
        return ((9 / mpmath.pi ** 2) ** k * (486 / (5 * mpmath.pi ** 4)) ** b
                * inv_p2 ** (-k) * inv_p4 ** (-b) * fin_k)


def d(k: int, m: int = 10**7, dps: int = 45):
    """d_k = prod over odd primes (1 - k/p^2) = (1 - k/9) d'_k, for k <= 8."""
    if not 1 <= k <= 8:
        raise ValueError("k must be in 1..8")
    with mpmath.workdps(dps):
        return (1 - mpmath.mpf(k) / 9) * d_prime(k, m, dps)


def c_small(l: int, m: int = 10**7, dps: int = 45):
    """c_l for l <= 6: sum_m binom(l, m) (-1)^(m-1) d_m (Section 2, l <= 6)."""
    if not 1 <= l <= 6:
        raise ValueError("l must be in 1..6")
    with mpmath.workdps(dps):
        return mpmath.fsum(math.comb(l, j) * (-1) ** (j - 1) * d(j, m, dps) for j in range(1, l + 1))


def _subset_counts(l: int):
    """N[s][r] = number of subsets I of {1..l} with |I| = s and |I mod 6| = r."""
    sizes = [sum(1 for k in range(1, l + 1) if k % 6 == res) for res in range(6)]
    N = [[0] * 7 for _ in range(l + 1)]
    N[0][0] = 1
    for n_res in sizes:
        nxt = [[0] * 7 for _ in range(l + 1)]
        for s in range(l + 1):
            for r in range(7):
                if not N[s][r]:
                    continue
                nxt[s][r] += N[s][r]  # no element of this residue class
                for j in range(1, n_res + 1):
                    if s + j <= l and r + 1 <= 6:
                        nxt[s + j][r + 1] += N[s][r] * math.comb(n_res, j)
        N = nxt
    return N


def c(l: int, m: int = 10**7, dps: int = 45):
    """c_l for 1 <= l <= 20 by equation (cell>6)."""
    if not 1 <= l <= 20:
        raise ValueError("l must be in 1..20")
    N = _subset_counts(l)
    with mpmath.workdps(dps):
        terms = []
        for s in range(1, l + 1):
            dp = d_prime(s, m, dps)
            for r in range(1, 7):
                if N[s][r]:
                    terms.append((-1) ** (s - 1) * N[s][r] * (1 - mpmath.mpf(r) / 9) * dp)
        return mpmath.fsum(terms)


def table(m: int = 10**7, dps: int = 45, lmax: int = 20):
    """Rows (l, 1 - c_l, c_l - c_(l-1)) for l = 1..lmax (mpf)."""
    rows, prev = [], mpmath.mpf(0)
    with mpmath.workdps(dps):
        for l in range(1, lmax + 1):
            cl = c(l, m, dps)
            rows.append((l, 1 - cl, cl - prev))
            prev = cl
    return rows


def moments(m: int = 10**7, dps: int = 45):
    """Mean and standard deviation of the least exponent, taking it to be at
    most 21 (c_21 := 1, as the section assumes); also the coefficients of
    E_S = mean/2 * S and sigma_S = sd / sqrt(2) * sqrt(S) for the odd n < S."""
    with mpmath.workdps(dps):
        rows = table(m, dps)
        probs = [p for _, _, p in rows] + [rows[-1][1]]  # P(k = 21) = 1 - c_20
        mean = mpmath.fsum((k + 1) * p for k, p in enumerate(probs))
        second = mpmath.fsum((k + 1) ** 2 * p for k, p in enumerate(probs))
        sd = mpmath.sqrt(second - mean ** 2)
        return {"mean": mean, "sd": sd, "E_S_coeff": mean / 2, "sigma_S_coeff": sd / mpmath.sqrt(2)}
