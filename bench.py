#!/usr/bin/env python3
"""Throughput of the verification path on one MI355X, per workload.

A step is one esq_verify_range call over the whole workload interval: the
sieve of Algorithm 1 and the least-k search of Algorithm 2 over every odd n of
the interval, with the aggregates (per-k counts, sum of k, maximum k,
record-setters, exceptions) reduced on the device.  Inputs are the interval
bounds; nothing is read from the host during the timed region.

The headline (`value`) is every odd n of [2^50 - 2^34 + 1, 2^50).  The line
also carries, under `configs`, each workload of the build with its own
throughput, roofline fraction and the oracle timed beside it on the host:
  odd_below_2pow22         all odd n in (1, 2^22], per-n output
  odd_2pow31_at_2pow40     2^31 odd n at 2^40
  odd_2pow33_below_2pow50  2^33 odd n just below 2^50 (the headline)
  batch_4096_intervals     4096 seeded intervals in one prepared batch
  served_poisson_2000      the seeded Poisson request stream through the server

Prints one JSON line (rank 0, N = 1).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs at 2.4 GHz.  VALU: the published fp32 vector peak, 157.3
# TFLOP/s, is 128 lanes x 2 flops per clock per CU, so 128 int32 lane-ops per
# clock per CU for the full-rate operations (funnel shifts and popcounts issue
# at half that rate; esq_measure_ceilings measures both).  LDS: 256 bytes per
# clock per CU (the measured ds_read_b64 rate exceeds the 128 bytes of CDNA3).
N_CU, CLK = 256, 2.4e9
VALU_PEAK = N_CU * 128 * CLK         # 7.86e13 lane-ops/s
LDS_PEAK = N_CU * 256 * CLK          # 1.57e14 B/s
HBM_PEAK = 8.0e12                    # B/s

# Work of the bit-sliced method per odd n:
#  LDS bytes: write the bitmap (1 bit), one 32-bit atomic OR per odd multiple
#  of p^2 for p >= 13 (density sum_{p>=13} 1/p^2 = 0.02241), read the bitmap
#  once (1 bit).
LDS_BYTES_PER_N = 0.125 + 4 * 0.02241 + 0.125
#  The sieve phase alone (Algorithm 1: bitmap init + marks, p >= 13 and the
#  large primes' 1.23e-4 hits per n): 0.125 + 4 * (0.02234 + 0.000123) B/n.
SIEVE_LDS_BYTES_PER_N = 0.125 + 4 * (0.02234 + 0.000123)
MARKS_PER_N = 0.02234 + 0.000123     # medium (17 <= p <= 4093) and large primes
#  VALU lane-ops: 6 per search step per 64-n word (two funnel shifts, two ANDs,
#  two popcounts) times the expected number of steps per word, 2.928, from the
#  probabilities of Table 2 (1 + sum_k P(some of 64 n unresolved after k)).
VALU_OPS_PER_N = 6 * 2.928 / 64

CONFIG_NAMES = ("odd_below_2pow22", "odd_2pow31_at_2pow40", "odd_2pow33_below_2pow50",
                "batch_4096_intervals", "served_poisson_2000")
HEADLINE = "odd_2pow33_below_2pow50"
TUNED = os.path.join(ROOT, "paper_2411_01964_amd", "tuned.json")

KERNEL_SRC = os.path.join(ROOT, "paper_2411_01964_amd", "csrc", "esq_kernels.hip")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_k_verify_odd_2pow33_below_2pow50.json")


def measured_traffic():
    """HBM bytes per launch of the segment kernel (summary, per-n and sieve)
    from the rocprofv3 counter runs recorded in profiles/ (FETCH_SIZE and
    WRITE_SIZE, scaled by the copy-probe factors) -- only while the kernel
    source is the one measured."""
    import hashlib
    try:
        with open(TRAFFIC) as f:
            t = json.load(f)
        with open(KERNEL_SRC, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != sha:
        return None
    out = {"summary": (t["fetch_kib_per_launch"] * t["fetch_factor"] +
                       t["write_kib_per_launch"] * t["write_factor"]) * 1024.0}
    if t.get("valu_insts_per_launch") is not None:
        out["valu_lane_ops"] = 64.0 * t["valu_insts_per_launch"]
    if t.get("sieve_fetch_kib_per_launch") is not None:
        out["sieve"] = (t["sieve_fetch_kib_per_launch"] * t["fetch_factor"] +
                        t["sieve_write_kib_per_launch"] * t["write_factor"]) * 1024.0
    if t.get("per_n_fetch_kib_per_launch") is not None:
        out["per_n"] = (t["per_n_fetch_kib_per_launch"] * t["fetch_factor"] +
                        t["per_n_write_kib_per_launch"] * t["write_factor"]) * 1024.0
    return out


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def n_odd_of(lo, hi):
    n0 = max(lo, 3) | 1
    return (hi - n0 + 1) // 2 if hi > n0 else 0


# ------------------------------------------------------------------ host side

def host_info():
    """Host cores as the process sees them, and the CPU model."""
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count() or 1
    return {"nproc": os.cpu_count() or 1, "affinity": affinity, "cpu_model": model}


def oracle_threads(host):
    """Threads for the oracle: every core the process may use, at most 16 (one
    GPU's share of the host cores of an eight-GPU node)."""
    return max(1, min(16, host["affinity"]))


def time_oracle(chunks, seconds, nthreads, label, host):
    """The oracle, as it stands, on seeded samples (an iterable of uint64 n
    arrays) until `seconds` of CPU work are done; returns a cpu_baseline."""
    import numpy as np

    import oracle

    count, dt = 0, 0.0
    for part in chunks:
        if dt >= seconds:
            break
        t0 = time.perf_counter()
        ks = oracle.mink_many(part, nthreads=nthreads)
        dt += time.perf_counter() - t0
        assert int(np.count_nonzero(ks == 0)) == 0
        count += len(part)
    return {"value": count / dt if dt else None, "unit": "odd n/s", "cores": nthreads,
            "kind": "oracle", "sample": "%d %s, trial division, %.1f s" % (count, label, dt),
            "nproc": host["nproc"], "cpu_model": host["cpu_model"]}


def random_chunks(seed, lo, hi, chunk, count=1 << 22):
    from paper_2411_01964_amd import workloads
    sample = workloads.random_odd(seed=seed, count=count, lo=lo, hi=hi)
    for s in range(0, len(sample), chunk):
        yield sample[s:s + chunk]


def per_interval_chunks(bounds, per, seed_base, chunk_intervals):
    """`per` seeded odd n inside each interval, `chunk_intervals` intervals
    at a time (the samples the parity tests store for the same workloads)."""
    import numpy as np

    from paper_2411_01964_amd import workloads
    for s in range(0, len(bounds), chunk_intervals):
        yield np.concatenate([workloads.random_odd(seed_base + i, per, a, b)
                              for i, (a, b) in enumerate(bounds[s:s + chunk_intervals], start=s)])


# ---------------------------------------------------------------- GPU side

def rooflines(n, kernel_s, ceil, kernel):
    """LDS (the metric's) and VALU rooflines of one segment-kernel launch over
    n odd n: algorithmic units per launch over the launch's duration."""
    lds_ach = LDS_BYTES_PER_N * n / kernel_s
    valu_ach = VALU_OPS_PER_N * n / kernel_s
    lds_meas = max(ceil["lds_write_b64_Bps"], ceil["lds_read_b64_Bps"])
    lds = {"bound": "lds", "achieved": lds_ach / 1e9, "peak": LDS_PEAK / 1e9, "unit": "GB/s",
           "frac": lds_ach / LDS_PEAK, "traffic": None, "kernel": kernel,
           "kernel_ms": kernel_s * 1e3, "algorithmic_bytes_per_n": LDS_BYTES_PER_N,
           "peak_measured": lds_meas / 1e9, "frac_measured": lds_ach / lds_meas}
    valu = {"bound": "alu", "achieved": valu_ach / 1e12, "peak": VALU_PEAK / 1e12,
            "unit": "Tlane-op/s", "frac": valu_ach / VALU_PEAK, "kernel": kernel,
            "kernel_ms": kernel_s * 1e3, "algorithmic_ops_per_n": VALU_OPS_PER_N,
            "peak_measured": ceil["valu_int32_ops_per_s"] / 1e12,
            "frac_measured": valu_ach / ceil["valu_int32_ops_per_s"]}
    return lds, valu


def run_range(lo, hi, steps, warmup, streams, per_n=False, prof_steps=20):
    """`warmup` untimed then `steps` timed esq_verify_range calls over [lo, hi)
    alternating over `streams` HIP streams; then up to prof_steps calls on one
    stream with the segment kernel's launch events (its duration for the
    roofline, and the one-stream time per step).  Every result is checked
    against the first."""
    import torch

    from paper_2411_01964_amd import esq

    n_odd = n_odd_of(lo, hi)
    ss = [torch.cuda.Stream() for _ in range(max(1, streams))]
    ref = esq.verify_range(lo, hi, per_n=per_n)            # reference result (untimed)
    for i in range(warmup):
        esq.verify_range_async(lo, hi, per_n=per_n, stream=ss[i % len(ss)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pend = [esq.verify_range_async(lo, hi, per_n=per_n, stream=ss[i % len(ss)])
            for i in range(steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for p in pend:
        r = p.result()
        assert r["status"] == 0 and sum(r["hist"]) == n_odd
        assert r["hist"] == ref["hist"] and r["records"] == ref["records"]
        if per_n:
            assert torch.equal(r["per_n"], ref["per_n"])
    del pend
    k = max(1, min(steps, prof_steps))
    esq.set_param("profile", 1)
    esq.profile_take()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(k):
        esq.verify_range_async(lo, hi, per_n=per_n)
    torch.cuda.synchronize()
    one = (time.perf_counter() - t1) / k
    seg_ms, launches = esq.profile_take()
    esq.set_param("profile", 0)
    return {"value": n_odd * steps / elapsed, "unit": "odd n/s", "n_odd": n_odd, "steps": steps,
            "warmup": warmup, "streams": len(ss), "ms_per_step": elapsed / steps * 1e3,
            "ms_per_step_one_stream": one * 1e3,
            "kernel_s": (seg_ms / max(launches, 1)) / 1e3}, ref


def sieve_phase(n, kernel_s, ph, ceil, traffic):
    """The segment kernel's time split by the phase clock, each phase against
    the ceiling that binds it: init (16-byte L2 reads of the two pattern
    tables, 16 bytes per region word) against the L2 read ceiling, marking
    (one ds_or_b32 per odd multiple of p^2, p >= 17) against the ds_or_b32
    ceiling, search (the algorithmic VALU operations, a third of them full
    rate, two thirds funnel shifts and popcounts) against the measured mix of
    those rates.  The sieve phase (init + marking) carries the paper's LDS
    traffic against the measured LDS peak."""
    from paper_2411_01964_amd import esq

    tot = max(1, sum(ph.values()))
    t_init = kernel_s * ph["init"] / tot
    t_mark = kernel_s * ph["mark"] / tot
    t_search = kernel_s * ph["search_or_store"] / tot
    S = 1 << esq.get_param("seg_log2")
    kh = esq.get_param("kh")
    rw_words = ((1 << (kh - 1)) if kh >= 7 else 64) // 64 + S // 64
    region = rw_words * 64
    l2_bytes = n / S * rw_words * 16
    marks = n * region / S * MARKS_PER_N
    mix = 1.0 / ((1 / ceil["valu_int32_ops_per_s"] + 1 / ceil["valu_alignbit_ops_per_s"] +
                  1 / ceil["valu_bcnt_ops_per_s"]) / 3)
    lds_meas = max(ceil["lds_write_b64_Bps"], ceil["lds_read_b64_Bps"])
    sieve_s = t_init + t_mark
    out = {
        "share_init": ph["init"] / tot, "share_mark": ph["mark"] / tot,
        "share_search": ph["search_or_store"] / tot,
        "ms": sieve_s * 1e3, "lds_bytes_per_n": SIEVE_LDS_BYTES_PER_N,
        "achieved_GBps": SIEVE_LDS_BYTES_PER_N * n / sieve_s / 1e9,
        "peak_measured_GBps": lds_meas / 1e9,
        "frac_measured": SIEVE_LDS_BYTES_PER_N * n / sieve_s / lds_meas,
        "frac_nominal": SIEVE_LDS_BYTES_PER_N * n / sieve_s / LDS_PEAK,
        "init": {"ms": t_init * 1e3, "bound": "l2 read", "l2_bytes": l2_bytes,
                 "achieved_GBps": l2_bytes / t_init / 1e9,
                 "ceiling_GBps": ceil["l2_read_Bps"] / 1e9,
                 "frac_of_ceiling": l2_bytes / t_init / ceil["l2_read_Bps"]},
        "mark": {"ms": t_mark * 1e3, "bound": "ds_or_b32", "marks": marks,
                 "achieved_GBps": 4 * marks / t_mark / 1e9,
                 "ceiling_GBps": ceil["lds_or_b32_Bps"] / 1e9,
                 "frac_of_ceiling": 4 * marks / t_mark / ceil["lds_or_b32_Bps"]},
        "search": {"ms": t_search * 1e3, "bound": "valu mix",
                   "achieved_Tops": VALU_OPS_PER_N * n / t_search / 1e12,
                   "ceiling_Tops": mix / 1e12,
                   "frac_of_ceiling": VALU_OPS_PER_N * n / t_search / mix},
    }
    if traffic and traffic.get("valu_lane_ops") is not None:
        out["issued_valu_Tops"] = traffic["valu_lane_ops"] / kernel_s / 1e12
    return out


def bench_per_n(lo, hi, n_odd, ref, steps=5):
    """The same interval in per-n mode: one least-k byte per odd n written to
    HBM (n_odd bytes per call).  The segment kernel's duration comes from the
    library's launch events; its bound is the HBM write of the bytes."""
    import torch

    from paper_2411_01964_amd import esq

    r = esq.verify_range(lo, hi, per_n=True)
    assert r["hist"] == ref["hist"] and r["records"] == ref["records"]
    # the first 2^24 bytes sum to the sum of least k over their n
    head = min(n_odd, 1 << 24)
    n0 = max(lo, 3) | 1
    part = esq.verify_range(lo, n0 + 2 * head)
    assert int(torch.sum(r["per_n"][:head], dtype=torch.int64)) == part["ksum"]
    del r
    esq.set_param("profile", 1)
    esq.profile_take()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = esq.verify_range(lo, hi, per_n=True)
        del r
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    seg_ms, launches = esq.profile_take()
    esq.set_param("profile", 0)
    k_s = seg_ms / max(launches, 1) / 1e3
    return {"odd_n_per_s": n_odd / wall, "ms_per_call": wall * 1e3, "kernel_ms": k_s * 1e3,
            "kernel_odd_n_per_s": n_odd / k_s, "block": esq.get_param("per_n_block"),
            "roofline": {"bound": "hbm", "achieved": n_odd / k_s / 1e9, "peak": 8000.0, "unit": "GB/s",
                         "frac": n_odd / k_s / HBM_PEAK, "traffic": None,
                         "kernel": "k_segment (per-n)"}}


def bench_sieve(lo, hi, steps=5):
    """Algorithm 1 alone over the same interval of odd m: one bit per odd m
    written to HBM.  The segment kernel's duration comes from the library's
    launch events; its bound is the HBM write of the bitmap."""
    import torch

    from paper_2411_01964_amd import esq

    m0, n, w = esq.sieve_segment(lo, hi)
    out_bytes = 8 * w.numel()
    esq.set_param("profile", 1)
    esq.profile_take()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        esq.sieve_segment(lo, hi, out=w)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    seg_ms, launches = esq.profile_take()
    esq.set_param("profile", 0)
    k_s = seg_ms / max(launches, 1) / 1e3
    del w
    return {"odd_m_per_s": n / wall, "ms_per_call": wall * 1e3, "kernel_ms": k_s * 1e3,
            "kernel_odd_m_per_s": n / k_s, "block": esq.get_param("sieve_block"),
            "seg_log2": esq.get_param("sieve_seg_log2"),
            "roofline": {"bound": "hbm", "achieved": out_bytes / k_s / 1e9, "peak": 8000.0, "unit": "GB/s",
                         "frac": out_bytes / k_s / HBM_PEAK, "traffic": None,
                         "kernel": "k_segment (sieve)"}}


def load_tuned(kind):
    """Knobs the autotuner chose for a workload kind (committed JSON), or {}."""
    try:
        with open(TUNED) as f:
            return dict(json.load(f).get(kind, {}).get("knobs", {}))
    except (OSError, ValueError):
        return {}


def bench_batched(steps, ceil):
    """Batched intervals: 4096 seeded intervals (lengths 2^16..2^28 odd n,
    starts in [2^30, 2^50)) in one prepared batch replayed as a hipGraph,
    against the plain path (one esq_verify_range per interval, back to back on
    one stream), with the knobs the autotuner chose for this workload.
    Results must agree exactly."""
    import torch

    from paper_2411_01964_amd import esq, tune, workloads

    lo, hi = workloads.batch_intervals(seed=4, count=4096)
    n_total = sum(n_odd_of(a, b) for a, b in zip(lo, hi))
    defaults = {k: esq.get_param(k) for k in ("seg_log2", "block", "medium_max", "items_per_wg", "stagger")}
    knobs = load_tuned("batch_4096_intervals")
    tune.apply(knobs)
    pb = esq.PreparedBatch(lo, hi)
    pb.launch(graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pb.launch(graph=True)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    batched = pb.results()
    pb.close()
    # the segment kernel's own duration: a prepared batch made while the
    # launch events are on, launched plainly
    esq.set_param("profile", 1)
    pbp = esq.PreparedBatch(lo, hi)
    esq.profile_take()
    for _ in range(steps):
        pbp.launch(graph=False)
    torch.cuda.synchronize()
    seg_ms, launches = esq.profile_take()
    esq.set_param("profile", 0)
    for x, y in zip(pbp.results(), batched):
        assert x["hist"] == y["hist"] and x["records"] == y["records"]
    pbp.close()
    tune.apply(defaults)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pend = [esq.verify_range_async(a, b) for a, b in zip(lo, hi)]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    plain = [p.result() for p in pend]
    for x, y in zip(batched, plain):
        assert x["hist"] == y["hist"] and x["records"] == y["records"]
    kernel_s = seg_ms / max(launches, 1) / 1e3
    lds, _ = rooflines(n_total, kernel_s, ceil, "k_segment (batch)")
    return {"intervals": len(lo), "odd_n": n_total, "knobs": knobs,
            "value": n_total / t_batch, "unit": "odd n/s",
            "batched_ms": t_batch * 1e3, "kernel_ms": kernel_s * 1e3,
            "plain_odd_n_per_s": n_total / t_plain, "plain_ms": t_plain * 1e3,
            "speedup": t_plain / t_batch, "identical": True, "roofline": lds}, (lo, hi)


def bench_served(ceil):
    """Served stream: Poisson arrivals (2000 req/s, seeded), lengths 2^12..2^30
    odd n, starts in [3, 2^50), half asking for per-n least k.  1 s warm-up
    plus 10 s measured; p50/p99 latency from arrival to completion.  Then the
    same requests all at once through the server (its capacity; one untimed
    pass first) and through the plain path (one esq_verify_range per request,
    in order); every served result (aggregates and records) equals the plain
    one."""
    import torch

    from paper_2411_01964_amd import esq, serve, workloads

    reqs = workloads.poisson_requests(seed=5, rate=2000.0, duration=11.0)
    done, wall, paced = serve.run_stream(reqs, n_streams=4, warmup_s=1.0, paced=True,
                                         keep_per_n=False)
    summ = [(r.result["hist"], r.result["records"], r.result["ksum"]) for r in done]
    del done
    # the capacity run: every request at once, after one untimed pass of the
    # same (the allocator's pool of per-n output slabs grows to the depth of
    # an unpaced stream on the first pass); both passes are checked
    summ_u = []
    for _ in range(2):
        done_u, wall_u, unpaced = serve.run_stream(reqs, n_streams=4, warmup_s=0.0, paced=False,
                                                   keep_per_n=False)
        summ_u.append([(r.result["hist"], r.result["records"], r.result["ksum"]) for r in done_u])
        del done_u
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_plain = 0
    plain = []
    for _, a, b, per_n in reqs:
        r = esq.verify_range(a, b, per_n=per_n)
        n_plain += r["n_odd"]
        plain.append((r["hist"], r["records"], r["ksum"]))
        del r
    t_plain = time.perf_counter() - t0
    assert summ == plain and summ_u[0] == plain and summ_u[1] == plain, \
        "served results differ from the plain path"
    cap = unpaced["odd_n"] / wall_u
    lds_ach = LDS_BYTES_PER_N * cap
    lds_meas = max(ceil["lds_write_b64_Bps"], ceil["lds_read_b64_Bps"])
    return {"requests": paced["requests"], "offered_odd_n_per_s": paced["odd_n"] / 11.0,
            "value": cap, "unit": "odd n/s",
            "p50_ms": paced["p50_ms"], "p99_ms": paced["p99_ms"],
            "served_paced_odd_n_per_s": paced["odd_n"] / wall,
            "served_capacity_odd_n_per_s": cap,
            "plain_odd_n_per_s": n_plain / t_plain, "batches": paced["batches"],
            "batches_unpaced": unpaced["batches"], "identical_to_plain": True,
            "roofline": {"bound": "lds", "achieved": lds_ach / 1e9, "peak": LDS_PEAK / 1e9,
                         "unit": "GB/s", "frac": lds_ach / LDS_PEAK,
                         "frac_measured": lds_ach / lds_meas, "traffic": None,
                         "kernel": "whole served stream, end to end (all kernels, host scheduling)"}}, reqs


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--streams", type=int, default=3,
                    help="steps alternate over this many HIP streams, so that one step's "
                         "setup kernels overlap another step's segment kernel")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="oracle seconds per workload for the CPU baselines")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--knobs", default="",
                    help="comma-separated name=value library knobs, e.g. seg_log2=17,block=512")
    ap.add_argument("--tune", action="store_true",
                    help="sweep the knobs on the workload first and use the fastest")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline workload (no other configs, batched or served)")
    ap.add_argument("--configs", default=",".join(CONFIG_NAMES[:2] + CONFIG_NAMES[3:]),
                    help="comma-separated workloads measured beside the headline")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (counter calibration)")
    args = ap.parse_args()

    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copied %d bytes" % args.copy_probe)
        return

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2411_01964_amd import esq, workloads

    host = host_info()
    nthreads = oracle_threads(host)
    lo, hi = workloads.CONFIGS[args.workload]
    n_odd = n_odd_of(lo, hi)
    log("init; host %s" % host)
    esq.init(0, max(hi + 64, (1 << 50) + (1 << 31)))
    if args.knobs:
        for kv in args.knobs.split(","):
            k, v = kv.split("=")
            esq.set_param(k.strip(), int(v))
    if args.tune:
        from paper_2411_01964_amd import tune
        best, t = tune.tune_range(lo, hi, reps=5)
        log("tuned: %s (%.3f ms)" % (best, t * 1e3))

    log("ceilings")
    ceil = esq.measure_ceilings()
    ceilings = {"lds_write_b64_GBps": ceil["lds_write_b64_Bps"] / 1e9,
                "lds_read_b64_GBps": ceil["lds_read_b64_Bps"] / 1e9,
                "lds_or_b32_GBps": ceil["lds_or_b32_Bps"] / 1e9,
                "valu_int32_Tops": ceil["valu_int32_ops_per_s"] / 1e12,
                "valu_alignbit_Tops": ceil["valu_alignbit_ops_per_s"] / 1e12,
                "valu_bcnt_Tops": ceil["valu_bcnt_ops_per_s"] / 1e12,
                "l2_read_GBps": ceil["l2_read_Bps"] / 1e9,
                "hbm_write_GBps": ceil["hbm_write_Bps"] / 1e9,
                "nominal_lds_GBps": LDS_PEAK / 1e9, "nominal_valu_Tops": VALU_PEAK / 1e12}

    # ---- the headline workload
    log("headline: %d warm-up + %d timed steps over %d odd n, %d stream(s)"
        % (args.warmup, args.steps, n_odd, args.streams))
    head, ref = run_range(lo, hi, args.steps, args.warmup, args.streams)
    log("%.4g odd n/s, %.4f ms/step (%.4f ms on one stream)"
        % (head["value"], head["ms_per_step"], head["ms_per_step_one_stream"]))
    seg_s = head["kernel_s"]
    roof, roof_valu = rooflines(n_odd, seg_s, ceil, "k_segment")
    traffic = (measured_traffic() if args.workload == HEADLINE else None) or {}
    roof["traffic"] = traffic.get("summary")
    if traffic.get("valu_lane_ops") is not None:
        issued = traffic["valu_lane_ops"] / seg_s
        roof_valu["issued"] = {"achieved": issued / 1e12, "frac": issued / VALU_PEAK,
                               "source": "SQ_INSTS_VALU of the committed counter run"}
    esq.set_param("phase_clock", 1)
    esq.phase_take()
    for _ in range(20):
        esq.verify_range_async(lo, hi)
    torch.cuda.synchronize()
    ph = esq.phase_take()
    esq.set_param("phase_clock", 0)
    phases = sieve_phase(n_odd, seg_s, ph, ceil, traffic)
    log("phases: %s" % phases)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline, headline (oracle, %d threads, ~%.0f s)" % (nthreads, args.cpu_seconds))
        import oracle
        oracle.mink_many(workloads.random_odd(seed=3, count=2, lo=lo, hi=hi), nthreads=1)
        cpu = time_oracle(random_chunks(31, lo, hi, 64 * nthreads), args.cpu_seconds, nthreads,
                          "seeded random odd n of the workload interval", host)

    log("per-n mode: %d bytes per call" % n_odd)
    per_n = bench_per_n(lo, hi, n_odd, ref)
    per_n["roofline"]["traffic"] = traffic.get("per_n")
    per_n["roofline"]["frac_of_write_ceiling"] = per_n["roofline"]["achieved"] * 1e9 / ceil["hbm_write_Bps"]
    log("sieve alone: %d bits per call" % n_odd)
    sieve = bench_sieve(lo, hi)
    sieve["roofline"]["traffic"] = traffic.get("sieve")
    sieve["roofline"]["frac_of_write_ceiling"] = sieve["roofline"]["achieved"] * 1e9 / ceil["hbm_write_Bps"]

    configs = {args.workload: dict(head, roofline=roof, cpu_baseline=cpu)}
    configs[args.workload].pop("kernel_s", None)
    configs[args.workload]["kernel_ms"] = seg_s * 1e3
    extra = set() if args.no_extras else {c.strip() for c in args.configs.split(",") if c.strip()}
    unknown = extra - set(CONFIG_NAMES)
    if unknown:
        raise SystemExit("unknown workloads: %s" % ", ".join(sorted(unknown)))
    if "odd_below_2pow22" in extra:
        import numpy as np

        import oracle
        # all odd n in (1, 2^22] with per-n output, the oracle over the whole interval
        a, b = workloads.CONFIGS["odd_below_2pow22"]
        log("odd_below_2pow22")
        c1, r1 = run_range(a, b, 50, max(args.warmup, 1), args.streams, per_n=True)
        l1, _ = rooflines(c1["n_odd"], c1.pop("kernel_s"), ceil, "k_segment (per-n)")
        cpu1 = None
        if not args.no_cpu_baseline:
            t0 = time.perf_counter()
            o = oracle.verify_range(a, b, per_n=True, nthreads=nthreads)
            dt = time.perf_counter() - t0
            assert np.array_equal(r1["per_n"].cpu().numpy(), o["per_n"])
            assert r1["hist"] == o["hist"] and r1["records"] == o["records"]
            cpu1 = {"value": c1["n_odd"] / dt, "unit": "odd n/s", "cores": nthreads,
                    "kind": "oracle", "sample": "the whole interval, %d odd n, trial division, "
                    "%.1f s (per-n bytes and aggregates equal the GPU's)" % (c1["n_odd"], dt),
                    "nproc": host["nproc"], "cpu_model": host["cpu_model"]}
        del r1
        configs["odd_below_2pow22"] = dict(c1, roofline=l1, cpu_baseline=cpu1)

    if "odd_2pow31_at_2pow40" in extra:
        a, b = workloads.CONFIGS["odd_2pow31_at_2pow40"]
        log("odd_2pow31_at_2pow40")
        c2, _ = run_range(a, b, 100, max(args.warmup, 6), args.streams)
        l2, _ = rooflines(c2["n_odd"], c2.pop("kernel_s"), ceil, "k_segment")
        cpu2 = None
        if not args.no_cpu_baseline:
            cpu2 = time_oracle(random_chunks(2, a, b, 1024 * nthreads), args.cpu_seconds, nthreads,
                               "seeded random odd n of the workload interval", host)
        configs["odd_2pow31_at_2pow40"] = dict(c2, roofline=l2, cpu_baseline=cpu2)

    if "batch_4096_intervals" in extra:
        log("batch_4096_intervals")
        c4, (blo, bhi) = bench_batched(5, ceil)
        if not args.no_cpu_baseline:
            c4["cpu_baseline"] = time_oracle(
                per_interval_chunks(list(zip(blo, bhi)), 64, 4000, 2 * nthreads), args.cpu_seconds,
                nthreads, "seeded odd n, 64 per interval", host)
        configs["batch_4096_intervals"] = c4

    if "served_poisson_2000" in extra:
        log("served_poisson_2000 (11 s paced, then unpaced, then plain)")
        c5, reqs = bench_served(ceil)
        if not args.no_cpu_baseline:
            c5["cpu_baseline"] = time_oracle(
                per_interval_chunks([(r[1], r[2]) for r in reqs], 16, 5000, 4 * nthreads),
                args.cpu_seconds, nthreads, "seeded odd n, 16 per request", host)
        configs["served_poisson_2000"] = c5

    r0 = ref
    served = configs.get("served_poisson_2000", {})
    out = {
        "metric": "odd n verified/sec near 2^50 (1 GPU)",
        "value": head["value"],
        "unit": "odd n/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "ms_per_step_one_stream": head["ms_per_step_one_stream"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "every odd n in [%d, %d) (%s)" % (lo, hi, args.workload),
            "n_odd": n_odd,
            "seg_log2": esq.get_param("seg_log2"),
            "kh": esq.get_param("kh"),
            "block": esq.get_param("block"),
            "medium_max": esq.get_param("medium_max"),
            "streams": head["streams"],
        },
        "roofline": roof,
        "roofline_valu": roof_valu,
        "cpu_baseline": cpu,
        "latency_p50_ms": served.get("p50_ms"),
        "latency_p99_ms": served.get("p99_ms"),
        "host": host,
        "ceilings": ceilings,
        "sieve_phase": phases,
        "per_n": per_n,
        "sieve": sieve,
        "configs": configs,
        "result": {"kmax_seen": r0["kmax_seen"], "ksum": r0["ksum"],
                   "records": r0["records"], "n_exceptions": r0["n_exceptions"]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
