"""Autotuner for the knobs that change speed but never results: segment
length (seg_log2), workgroup size (block; waves per CU follow from it and the
LDS a segment needs), the medium/large prime cut-over (medium_max), the start
stagger of co-resident workgroups and, for batches, work items per resident
workgroup (items_per_wg).

Each candidate is timed with whole launches (a prepared batch, or
esq_verify_range calls) on one stream after a warm-up launch; its results must
equal the first candidate's.  The best setting per workload kind is kept in
tuned.json beside this file, which bench.py reads:

    python -m paper_2411_01964_amd.tune batch      # the 4096-interval batch
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

import torch

from . import esq

SPACE = {
    "seg_log2": (16, 17, 18, 19),
    "block": (256, 512, 1024),
    "medium_max": (2047, 4095, 8191),
    "stagger": (0, 72),
}
BATCH_SPACE = dict(SPACE, items_per_wg=(1, 2, 4, 8))
TUNED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def apply(knobs: dict):
    for k, v in knobs.items():
        esq.set_param(k, int(v))


def _time_call(fn, reps):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _sweep(space, run, verbose):
    """run(knobs) -> (seconds, comparable result); returns the sorted table."""
    table, ref = [], None
    names = list(space)
    for combo in itertools.product(*(space[n] for n in names)):
        knobs = dict(zip(names, combo))
        apply(knobs)
        try:
            t, res = run(knobs)
        except esq.EsqError as e:      # e.g. a segment too large for LDS
            if verbose:
                print("tune %s skipped: %s" % (knobs, e), flush=True)
            continue
        if ref is None:
            ref = res
        assert res == ref, "results depend on the knobs %s" % knobs
        table.append((t, knobs))
        if verbose:
            print("tune %s %.3f ms" % (knobs, t * 1e3), flush=True)
    table.sort(key=lambda x: x[0])
    apply(table[0][1])
    return table


def tune_range(lo, hi, reps=5, space=SPACE, verbose=False):
    """Best knobs for esq_verify_range over [lo, hi); returns (knobs, seconds)."""
    def run(knobs):
        r = esq.verify_range(lo, hi)
        t = _time_call(lambda: esq.verify_range_async(lo, hi), reps)
        return t, (r["hist"], r["records"])
    table = _sweep(space, run, verbose)
    return table[0][1], table[0][0]


def tune_batch(los, his, reps=3, space=BATCH_SPACE, verbose=False):
    """Best knobs for a prepared batch of intervals; returns (knobs, seconds,
    table of (seconds, knobs) in increasing time)."""
    def run(knobs):
        pb = esq.PreparedBatch(los, his)
        try:
            t = _time_call(lambda: pb.launch(graph=True), reps)
            res = pb.results()
        finally:
            pb.close()
        return t, [(r["hist"], r["records"]) for r in res]
    table = _sweep(space, run, verbose)
    return table[0][1], table[0][0], table


def store(kind, knobs, seconds, table=None, workload=""):
    """Keep the chosen knobs of a workload kind in tuned.json."""
    data = {}
    try:
        with open(TUNED) as f:
            data = json.load(f)
    except (OSError, ValueError):
        pass
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    entry = {"knobs": knobs, "ms": seconds * 1e3, "workload": workload,
             "device": "%s, %d CUs" % (props.name, props.multi_processor_count)}
    if table:
        entry["fastest"] = [{"ms": t * 1e3, "knobs": k} for t, k in table[:8]]
        entry["slowest_ms"] = table[-1][0] * 1e3
        entry["candidates"] = len(table)
    data[kind] = entry
    tmp = TUNED + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, TUNED)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("kind", choices=["batch"])
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    from . import workloads
    esq.init(0, (1 << 50) + (1 << 31))
    if args.kind == "batch":
        lo, hi = workloads.batch_intervals(seed=4, count=4096)
        knobs, t, table = tune_batch(lo, hi, reps=args.reps, verbose=True)
        store("batch_4096_intervals", knobs, t, table,
              "4096 seeded intervals (lengths 2^16..2^28 odd n, starts in [2^30, 2^50)), "
              "one prepared batch replayed as a hipGraph")
        print("batch: %s %.3f ms (of %d candidates)" % (knobs, t * 1e3, len(table)), flush=True)


if __name__ == "__main__":
    sys.exit(main())
