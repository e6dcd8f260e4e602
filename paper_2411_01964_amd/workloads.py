"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  This module draws numbers only; it holds none of the method's
arithmetic (no squarefreeness, no least-k logic).

The workload class is the paper's own: whole intervals of odd integers
(Section 3, both algorithms take an interval [start, end)).  No dataset is
involved; the configurations below place such intervals at other positions
and sizes.
"""
from __future__ import annotations

import math

import numpy as np

# name -> (lo, hi); every odd n in [lo, hi) with n >= 3 is examined
CONFIGS = {
    # all odd n in (1, 2^22]: 2,097,151 odd integers
    "odd_below_2pow22": (3, (1 << 22) + 1),
    # one contiguous interval of 2^31 odd integers at 2^40
    "odd_2pow31_at_2pow40": ((1 << 40) + 1, (1 << 40) + (1 << 32)),
    # the last 2^34 integers below the paper's bound 2^50: 2^33 odd integers
    "odd_2pow33_below_2pow50": ((1 << 50) - (1 << 34) + 1, 1 << 50),
}


def random_odd(seed: int, count: int, lo: int, hi: int) -> np.ndarray:
    """count odd integers drawn uniformly from [lo, hi) (uint64, sorted)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    first = lo | 1
    n_odd = (hi - first + 1) // 2
    idx = rng.integers(0, n_odd, size=count, dtype=np.uint64)
    return np.sort(np.uint64(first) + np.uint64(2) * idx).astype(np.uint64)


def random_windows(seed: int, count: int, width: int, lo: int, hi: int):
    """count windows [a, a + 2*width) of `width` odd integers inside [lo, hi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    first = lo | 1
    n_odd = (hi - first + 1) // 2
    starts = rng.integers(0, n_odd - width, size=count, dtype=np.uint64)
    return [(int(first + 2 * int(s)), int(first + 2 * int(s) + 2 * width)) for s in sorted(starts)]


def batch_intervals(seed: int = 4, count: int = 4096, log2_len=(16, 28),
                    start_range=(1 << 30, 1 << 50)):
    """Intervals of uneven length and position: length L = floor(2^U) odd
    integers with U ~ Uniform(log2_len), start uniform over the odd integers
    of start_range.  Returns (lo, hi) arrays of Python ints."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(log2_len[0], log2_len[1], size=count)
    lengths = np.floor(np.exp2(u)).astype(np.int64)
    a, b = start_range
    starts = rng.integers(a // 2, b // 2, size=count, dtype=np.int64) * 2 + 1
    lo = [int(s) for s in starts]
    hi = [int(s) + 2 * int(L) for s, L in zip(starts, lengths)]
    return lo, hi


def poisson_requests(seed: int = 5, rate: float = 2000.0, duration: float = 11.0,
                     log2_len=(12, 30), start_range=(3, 1 << 50)):
    """A Poisson stream of interval queries: exponential gaps of mean
    1/rate seconds, lengths floor(2^U) odd integers with U ~ Uniform(log2_len),
    start uniform over odd integers, and a per-request mode drawn
    Bernoulli(0.5): True = per-n least k wanted, False = summary only.
    Returns a list of (t_arrival_s, lo, hi, per_n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out, t = [], 0.0
    a, b = start_range
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        L = int(math.floor(2.0 ** float(rng.uniform(*log2_len))))
        s = int(rng.integers(a // 2, b // 2)) * 2 + 1
        out.append((t, s, s + 2 * L, bool(rng.random() < 0.5)))
    return out
