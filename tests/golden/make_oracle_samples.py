#!/usr/bin/env python3
"""Write the stored oracle results that the full-size GPU parity tests compare
against.  This script calls only the oracle (``oracle/``) and the seeded input
generators (``paper_2411_01964_amd/workloads.py``, which hold none of the
method's arithmetic); no value here comes from the GPU path.

Each sample is a seeded set of odd n drawn from one of the workloads, with the
oracle's least k of every n (Algorithm 2, Section 3; trial division of
n - 2^k by odd prime squares):

  cfg2_random      2^20 odd n, uniform in [2^40 + 1, 2^40 + 2^32), seed 2
  cfg2_windows     64 windows of 2^16 consecutive odd n there, seed 2: every
                   n's least k, and each window's aggregates (Section 3,
                   "Collecting the results"; Tables 3 and 4)
  cfg3_random      2^20 odd n, uniform in [2^50 - 2^34 + 1, 2^50), seed 3
  cfg3_windows     16 windows of 2^12 consecutive odd n there, seed 3
  cfg4_sample      64 odd n inside each of the 4096 intervals of the batched
                   workload (seed 4), interval i drawn with seed 4000 + i
  cfg5_sample      the first 300 requests of the served Poisson stream
                   (seed 5): 16 odd n per request (seed 5000 + i), and every
                   n of the requests of at most 2^13 odd n in full, with
                   their aggregates

Files: <name>.json (what was drawn and how, the SHA-256 of the drawn n, the
aggregates) and <name>.k.xz (the least k bytes, in the order of the drawn n,
lzma-compressed).  Run from the repository root:

    python tests/golden/make_oracle_samples.py [name ...] [--threads N]

Samples whose files exist are skipped (delete them to recompute).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import lzma
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2411_01964_amd import workloads  # noqa: E402

OUT = os.path.join(HERE, "oracle_samples")

CFG2 = workloads.CONFIGS["odd_2pow31_at_2pow40"]
CFG3 = workloads.CONFIGS["odd_2pow33_below_2pow50"]


def sha_n(ns) -> str:
    return hashlib.sha256(np.ascontiguousarray(np.asarray(ns, dtype="<u8")).tobytes()).hexdigest()


def random_sample(name, seed, lo, hi, count):
    return {"kind": "random_odd", "seed": seed, "lo": lo, "hi": hi, "count": count}


def windows_sample(name, seed, lo, hi, count, width):
    return {"kind": "windows", "seed": seed, "lo": lo, "hi": hi, "count": count, "width": width}


SAMPLES = {
    "cfg2_random": random_sample("cfg2_random", 2, *CFG2, 1 << 20),
    "cfg2_windows": windows_sample("cfg2_windows", 2, *CFG2, 64, 1 << 16),
    "cfg3_random": random_sample("cfg3_random", 3, *CFG3, 1 << 20),
    "cfg3_windows": windows_sample("cfg3_windows", 3, *CFG3, 16, 1 << 12),
    "cfg4_sample": {"kind": "batch", "seed": 4, "count": 4096, "per_interval": 64, "seed_base": 4000},
    "cfg5_sample": {"kind": "served", "seed": 5, "rate": 2000.0, "duration": 11.0, "requests": 300,
                    "per_request": 16, "seed_base": 5000, "full_max_odd": 1 << 13},
}


def draw(spec):
    """The n of a sample in stored order, plus per-part bounds:
    (ns uint64 array, parts [(lo, hi, start, stop, full)])."""
    kind = spec["kind"]
    if kind == "random_odd":
        ns = workloads.random_odd(spec["seed"], spec["count"], spec["lo"], spec["hi"])
        return ns, []
    if kind == "windows":
        wins = workloads.random_windows(spec["seed"], spec["count"], spec["width"], spec["lo"], spec["hi"])
        chunks, parts, pos = [], [], 0
        for a, b in wins:
            n = np.arange(a | 1, b, 2, dtype=np.uint64)
            chunks.append(n)
            parts.append((a, b, pos, pos + n.size, True))
            pos += n.size
        return np.concatenate(chunks), parts
    if kind == "batch":
        lo, hi = workloads.batch_intervals(seed=spec["seed"], count=spec["count"])
        chunks, parts, pos = [], [], 0
        for i, (a, b) in enumerate(zip(lo, hi)):
            n = workloads.random_odd(spec["seed_base"] + i, spec["per_interval"], a, b)
            chunks.append(n)
            parts.append((a, b, pos, pos + n.size, False))
            pos += n.size
        return np.concatenate(chunks), parts
    if kind == "served":
        reqs = workloads.poisson_requests(seed=spec["seed"], rate=spec["rate"],
                                          duration=spec["duration"])[:spec["requests"]]
        chunks, parts, pos = [], [], 0
        for i, (_, a, b, _) in enumerate(reqs):
            n_odd = (b - (max(a, 3) | 1) + 1) // 2
            if n_odd <= spec["full_max_odd"]:
                n = np.arange(max(a, 3) | 1, b, 2, dtype=np.uint64)
                full = True
            else:
                n = workloads.random_odd(spec["seed_base"] + i, spec["per_request"], a, b)
                full = False
            chunks.append(n)
            parts.append((a, b, pos, pos + n.size, full))
            pos += n.size
        return np.concatenate(chunks), parts
    raise ValueError(kind)


def make(name, threads):
    spec = SAMPLES[name]
    js = os.path.join(OUT, name + ".json")
    kx = os.path.join(OUT, name + ".k.xz")
    if os.path.exists(js) and os.path.exists(kx):
        print("%s: exists, skipped" % name, flush=True)
        return
    t0 = time.time()
    ns, parts = draw(spec)
    k = np.zeros(ns.size, dtype=np.uint8)
    step = 1 << 14
    for s in range(0, ns.size, step):
        k[s:s + step] = oracle.mink_many(ns[s:s + step], nthreads=threads)
        if (s // step) % 16 == 0:
            print("%s: %d / %d n (%.0f s)" % (name, s + min(step, ns.size - s), ns.size, time.time() - t0),
                  flush=True)
    meta = dict(spec)
    meta.update({"name": name, "n_count": int(ns.size), "sha256_n": sha_n(ns),
                 "hist": np.bincount(k, minlength=65).astype(int).tolist(),
                 "written_by": "tests/golden/make_oracle_samples.py (oracle.mink_many, "
                               "oracle.verify_range)"})
    full_parts = []
    for a, b, start, stop, full in parts:
        if not full:
            continue
        o = oracle.verify_range(a, b, per_n=True, nthreads=threads)
        assert np.array_equal(o["per_n"], k[start:stop]), (name, a, b)
        full_parts.append({"lo": a, "hi": b, "start": start, "stop": stop, "hist": o["hist"],
                           "ksum": o["ksum"], "kmax_seen": o["kmax_seen"], "records": o["records"],
                           "n_exceptions": o["n_exceptions"]})
    if full_parts:
        meta["full"] = full_parts
    meta["seconds"] = round(time.time() - t0, 1)
    meta["threads"] = threads
    os.makedirs(OUT, exist_ok=True)
    with lzma.open(kx + ".tmp", "wb", preset=9 | lzma.PRESET_EXTREME) as f:
        f.write(k.tobytes())
    os.replace(kx + ".tmp", kx)
    with open(js + ".tmp", "w") as f:
        json.dump(meta, f, indent=1)
        f.write("\n")
    os.replace(js + ".tmp", js)
    print("%s: %d n in %.0f s" % (name, ns.size, time.time() - t0), flush=True)


def load(name):
    """(meta dict, ns uint64 array, k uint8 array, parts) of a stored sample;
    the drawn n are regenerated and checked against the stored SHA-256.
    parts: per window, batch interval or request, (lo, hi, start, stop,
    full) -- its n are ns[start:stop]; full = every odd n of [lo, hi)."""
    with open(os.path.join(OUT, name + ".json")) as f:
        meta = json.load(f)
    with lzma.open(os.path.join(OUT, name + ".k.xz"), "rb") as f:
        k = np.frombuffer(f.read(), dtype=np.uint8)
    ns, parts = draw(SAMPLES[name])
    assert sha_n(ns) == meta["sha256_n"], "the seeded generator no longer draws the stored n"
    assert k.size == ns.size
    return meta, ns, k, parts


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("names", nargs="*", default=list(SAMPLES))
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    for name in args.names:
        make(name, args.threads)


if __name__ == "__main__":
    main()
