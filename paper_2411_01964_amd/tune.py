"""Autotuner for the knobs that change speed but never results: segment
length (seg_log2), workgroup size (block; waves per CU follow from it and the
LDS a segment needs), the medium/large prime cut-over (medium_max) and, for
batches, work items per resident workgroup (items_per_wg).

Each candidate is timed with HIP events around the segment kernel (the
library's "profile" knob) plus the wall clock of whole calls; the best
setting per (device, workload kind, magnitude) is cached as JSON.
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time

import torch

from . import esq

SPACE = {
    "seg_log2": (16, 17, 18, 19),
    "block": (128, 256, 512, 1024),
    "medium_max": (2047, 4095, 8191),
}
BATCH_SPACE = dict(SPACE, items_per_wg=(1, 2, 4, 8))
CACHE = os.path.join(os.path.expanduser("~"), ".cache", "esq", "tune.json")


def _key(kind, lo, hi):
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    mag = int(math.log2(max(hi, 2)))
    return "%s|%d|%s|%s|2^%d" % (props.name, props.multi_processor_count,
                                 torch.version.hip, kind, mag)


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


def tune_range(lo, hi, reps=5, space=SPACE, verbose=False):
    """Best knobs for esq_verify_range over [lo, hi); returns (knobs, seconds)."""
    best = None
    ref = None
    names = list(space)
    for combo in itertools.product(*(space[n] for n in names)):
        knobs = dict(zip(names, combo))
        apply(knobs)
        r = esq.verify_range(lo, hi)
        if ref is None:
            ref = r
        assert r["hist"] == ref["hist"] and r["records"] == ref["records"]
        t = _time_call(lambda: esq.verify_range_async(lo, hi), reps)
        if verbose:
            print("tune", knobs, "%.3f ms" % (t * 1e3), flush=True)
        if best is None or t < best[1]:
            best = (knobs, t)
    apply(best[0])
    return best


def tune_batch(los, his, reps=3, space=BATCH_SPACE, verbose=False):
    """Best knobs for a prepared batch of intervals; returns (knobs, seconds)."""
    best = None
    ref = None
    names = list(space)
    for combo in itertools.product(*(space[n] for n in names)):
        knobs = dict(zip(names, combo))
        apply(knobs)
        pb = esq.PreparedBatch(los, his)
        try:
            t = _time_call(lambda: pb.launch(graph=False), reps)
            res = pb.results()
        finally:
            pb.close()
        if ref is None:
            ref = res
        assert all(a["hist"] == b["hist"] and a["records"] == b["records"] for a, b in zip(res, ref))
        if verbose:
            print("tune", knobs, "%.3f ms" % (t * 1e3), flush=True)
        if best is None or t < best[1]:
            best = (knobs, t)
    apply(best[0])
    return best


def cached(kind, lo, hi):
    try:
        with open(CACHE) as f:
            return json.load(f).get(_key(kind, lo, hi))
    except (OSError, ValueError):
        return None


def store(kind, lo, hi, knobs, seconds):
    data = {}
    try:
        with open(CACHE) as f:
            data = json.load(f)
    except (OSError, ValueError):
        pass
    data[_key(kind, lo, hi)] = {"knobs": knobs, "seconds": seconds}
    os.makedirs(os.path.dirname(CACHE), exist_ok=True)
    with open(CACHE, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
