#!/usr/bin/env python3
"""Throughput of the verification path on one MI355X.

A step is one esq_verify_range call over the whole workload interval: the
sieve of Algorithm 1 and the least-k search of Algorithm 2 over every odd n of
the interval, with the aggregates (per-k counts, sum of k, maximum k,
record-setters, exceptions) reduced on the device.  Inputs are the interval
bounds; nothing is read from the host during the timed region.

Prints one JSON line (rank 0, N = 1).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs at 2.4 GHz.  VALU: the published fp32 vector peak, 157.3
# TFLOP/s, is 128 lanes x 2 flops per clock per CU, so 128 int32 lane-ops per
# clock per CU for the full-rate operations (funnel shifts, popcounts and
# three-operand shift-adds issue at half that rate; esq_measure_ceilings and
# the benchmark's ceilings block measure both).  LDS: 256 bytes per clock per
# CU for reads (the measured ds_read_b64 rate exceeds the 128 bytes of CDNA3).
N_CU, CLK = 256, 2.4e9
VALU_PEAK = N_CU * 128 * CLK         # 7.86e13 lane-ops/s
LDS_PEAK = N_CU * 256 * CLK          # 1.57e14 B/s

# Work of the bit-sliced method per odd n:
#  LDS bytes: write the bitmap (1 bit), one 32-bit atomic OR per odd multiple
#  of p^2 for p >= 13 (density sum_{p>=13} 1/p^2 = 0.02241), read the bitmap
#  once (1 bit).
LDS_BYTES_PER_N = 0.125 + 4 * 0.02241 + 0.125
#  The sieve phase alone (Algorithm 1: bitmap init + marks, p >= 13 and the
#  large primes' 1.23e-4 hits per n): 0.125 + 4 * (0.02234 + 0.000123) B/n.
SIEVE_LDS_BYTES_PER_N = 0.125 + 4 * (0.02234 + 0.000123)
#  VALU lane-ops: 6 per search step per 64-n word (two funnel shifts, two ANDs,
#  two popcounts) times the expected number of steps per word, 2.928, from the
#  probabilities of Table 2 (1 + sum_k P(some of 64 n unresolved after k)).
VALU_OPS_PER_N = 6 * 2.928 / 64


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


def cpu_baseline(lo, hi, seconds, nthreads):
    """The oracle, as it stands, on a bounded seeded sample of the workload."""
    import numpy as np

    import oracle
    from paper_2411_01964_amd import workloads

    oracle.mink_many(workloads.random_odd(seed=3, count=2, lo=lo, hi=hi), nthreads=1)  # prime list
    # chunks of a seeded sample until the target time is reached
    sample = workloads.random_odd(seed=31, count=1 << 22, lo=lo, hi=hi)
    count, dt, chunk = 0, 0.0, 64 * nthreads
    while dt < seconds and count < len(sample):
        part = sample[count:count + chunk]
        t0 = time.perf_counter()
        ks = oracle.mink_many(part, nthreads=nthreads)
        dt += time.perf_counter() - t0
        assert int(np.count_nonzero(ks == 0)) == 0
        count += len(part)
    return {
        "value": count / dt,
        "unit": "odd n/s",
        "cores": nthreads,
        "kind": "oracle",
        "sample": "%d seeded random odd n of the workload interval, trial division, %.1f s"
                  % (count, dt),
    }


def bench_batched(steps):
    """Batched intervals: 4096 seeded intervals (lengths 2^16..2^28 odd n, starts in
    [2^30, 2^50)) in one prepared batch replayed as a hipGraph, against the
    plain path (one esq_verify_range per interval, back to back on one
    stream).  Results must agree exactly."""
    import torch

    from paper_2411_01964_amd import esq, workloads

    lo, hi = workloads.batch_intervals(seed=4, count=4096)
    n_total = sum(((b - (max(a, 3) | 1) + 1) // 2) for a, b in zip(lo, hi))
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
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pend = [esq.verify_range_async(a, b) for a, b in zip(lo, hi)]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    plain = [p.result() for p in pend]
    for x, y in zip(batched, plain):
        assert x["hist"] == y["hist"] and x["records"] == y["records"]
    return {"intervals": len(lo), "odd_n": n_total,
            "batched_odd_n_per_s": n_total / t_batch, "batched_ms": t_batch * 1e3,
            "plain_odd_n_per_s": n_total / t_plain, "plain_ms": t_plain * 1e3,
            "speedup": t_plain / t_batch, "identical": True}


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
            "kernel_odd_n_per_s": n_odd / k_s,
            "roofline": {"bound": "hbm", "achieved": n_odd / k_s / 1e9, "peak": 8000.0, "unit": "GB/s",
                         "frac": n_odd / k_s / 8e12, "traffic": None,
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
            "kernel_odd_m_per_s": n / k_s,
            "roofline": {"bound": "hbm", "achieved": out_bytes / k_s / 1e9, "peak": 8000.0, "unit": "GB/s",
                         "frac": out_bytes / k_s / 8e12, "traffic": None,
                         "kernel": "k_segment (sieve)"}}


def bench_served():
    """Served stream: Poisson arrivals (2000 req/s, seeded), lengths 2^12..2^30
    odd n, starts in [3, 2^50), half asking for per-n least k.  1 s warm-up
    plus 10 s measured; p50/p99 latency from arrival to completion.  Then the
    same requests all at once through the server (its capacity) and through
    the plain path (one esq_verify_range per request, in order)."""
    import torch

    from paper_2411_01964_amd import esq, serve, workloads

    reqs = workloads.poisson_requests(seed=5, rate=2000.0, duration=11.0)
    _, wall, paced = serve.run_stream(reqs, n_streams=4, warmup_s=1.0, paced=True,
                                      keep_per_n=False)
    _, wall_u, unpaced = serve.run_stream(reqs, n_streams=4, warmup_s=0.0, paced=False,
                                          keep_per_n=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_plain = 0
    for _, a, b, per_n in reqs:
        r = esq.verify_range(a, b, per_n=per_n)
        n_plain += r["n_odd"]
        del r
    t_plain = time.perf_counter() - t0
    return {"requests": paced["requests"], "offered_odd_n_per_s": paced["odd_n"] / 11.0,
            "p50_ms": paced["p50_ms"], "p99_ms": paced["p99_ms"],
            "served_paced_odd_n_per_s": paced["odd_n"] / wall,
            "served_capacity_odd_n_per_s": unpaced["odd_n"] / wall_u,
            "plain_odd_n_per_s": n_plain / t_plain, "batches": paced["batches"]}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="odd_2pow33_below_2pow50")
    ap.add_argument("--streams", type=int, default=3,
                    help="steps alternate over this many HIP streams, so that one step's "
                         "setup kernels overlap another step's segment kernel")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--knobs", default="",
                    help="comma-separated name=value library knobs, e.g. seg_log2=17,block=512")
    ap.add_argument("--tune", action="store_true",
                    help="sweep the knobs on the workload first and use the fastest")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched (4096 intervals) and served (Poisson) measurements")
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

    lo, hi = workloads.CONFIGS[args.workload]
    n0 = max(lo, 3) | 1
    n_odd = (hi - n0 + 1) // 2
    log("init")
    esq.init(0, hi + 64)
    if args.knobs:
        for kv in args.knobs.split(","):
            k, v = kv.split("=")
            esq.set_param(k.strip(), int(v))
    if args.tune:
        from paper_2411_01964_amd import tune
        best, t = tune.tune_range(lo, hi, reps=5)
        log("tuned: %s (%.3f ms)" % (best, t * 1e3))
    streams = [torch.cuda.Stream() for _ in range(max(1, args.streams))]
    # warm-up runs on the same streams as the timed steps (a stream's first
    # call grows the library's scratch pool for that stream)
    n_warm = max(args.warmup, 2 * len(streams))
    log("warmup x%d over %d odd n" % (n_warm, n_odd))
    warm = [esq.verify_range_async(lo, hi, stream=streams[i % len(streams)]) for i in range(n_warm)]
    ref = warm[-1].result()
    log("timed x%d over %d stream(s)" % (args.steps, len(streams)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pend = [esq.verify_range_async(lo, hi, stream=streams[i % len(streams)])
            for i in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = [p.result() for p in pend]
    for r in res:
        assert r["status"] == 0 and sum(r["hist"]) == n_odd
        if ref is not None:
            assert r["hist"] == ref["hist"] and r["records"] == ref["records"]
    elapsed = t1 - t0
    value = n_odd * args.steps / elapsed
    log("%.3f s for %d steps -> %.4g odd n/s" % (elapsed, args.steps, value))

    # segment-kernel duration for the roofline: a separate pass on one stream,
    # so that no other step's kernels share the device during a timed launch
    prof_steps = min(args.steps, 20)
    esq.set_param("profile", 1)
    esq.profile_take()
    for _ in range(prof_steps):
        esq.verify_range_async(lo, hi)
    torch.cuda.synchronize()
    seg_ms, launches = esq.profile_take()
    esq.set_param("profile", 0)

    seg_avg_s = (seg_ms / max(launches, 1)) / 1e3
    valu_ach = VALU_OPS_PER_N * n_odd / seg_avg_s
    lds_ach = LDS_BYTES_PER_N * n_odd / seg_avg_s
    roof_valu = {"bound": "alu", "achieved": valu_ach / 1e12, "peak": VALU_PEAK / 1e12,
                 "unit": "Tlane-op/s", "frac": valu_ach / VALU_PEAK, "traffic": None,
                 "kernel": "k_segment", "kernel_ms": seg_avg_s * 1e3}
    roof_lds = {"bound": "lds", "achieved": lds_ach / 1e9, "peak": LDS_PEAK / 1e9,
                "unit": "GB/s", "frac": lds_ach / LDS_PEAK, "traffic": None,
                "kernel": "k_segment", "kernel_ms": seg_avg_s * 1e3}
    roof, alt = (roof_valu, roof_lds) if roof_valu["frac"] >= roof_lds["frac"] else (roof_lds, roof_valu)
    traffic = (measured_traffic() if args.workload == "odd_2pow33_below_2pow50" else None) or {}
    roof["traffic"] = traffic.get("summary")
    alt["traffic"] = traffic.get("summary")
    if traffic.get("valu_lane_ops") is not None:
        # every VALU instruction the kernel issued (SQ_INSTS_VALU x 64 lanes),
        # not only the search's algorithmic ones
        issued = traffic["valu_lane_ops"] / seg_avg_s
        roof_valu["issued"] = {"achieved": issued / 1e12, "frac": issued / VALU_PEAK,
                               "source": "SQ_INSTS_VALU of the committed counter run"}

    # measured ceilings (microbenchmarks) and the kernel's time per phase
    ceil = esq.measure_ceilings()
    esq.set_param("phase_clock", 1)
    esq.phase_take()
    for _ in range(prof_steps):
        esq.verify_range_async(lo, hi)
    torch.cuda.synchronize()
    ph = esq.phase_take()
    esq.set_param("phase_clock", 0)
    tot = max(1, sum(ph.values()))
    sieve_s = seg_avg_s * (ph["init"] + ph["mark"]) / tot
    lds_peak = max(ceil["lds_write_b64_Bps"], ceil["lds_read_b64_Bps"])
    sieve_phase = {
        "share_init": ph["init"] / tot, "share_mark": ph["mark"] / tot, "share_search": ph["search_or_store"] / tot,
        "ms": sieve_s * 1e3, "lds_bytes_per_n": SIEVE_LDS_BYTES_PER_N,
        "achieved_GBps": SIEVE_LDS_BYTES_PER_N * n_odd / sieve_s / 1e9,
        "peak_measured_GBps": lds_peak / 1e9,
        "frac_measured": SIEVE_LDS_BYTES_PER_N * n_odd / sieve_s / lds_peak,
        "frac_nominal": SIEVE_LDS_BYTES_PER_N * n_odd / sieve_s / LDS_PEAK,
    }
    ceilings = {"lds_write_b64_GBps": ceil["lds_write_b64_Bps"] / 1e9,
                "lds_read_b64_GBps": ceil["lds_read_b64_Bps"] / 1e9,
                "lds_or_b32_GBps": ceil["lds_or_b32_Bps"] / 1e9,
                "valu_int32_Tops": ceil["valu_int32_ops_per_s"] / 1e12,
                "valu_alignbit_Tops": ceil["valu_alignbit_ops_per_s"] / 1e12,
                "valu_bcnt_Tops": ceil["valu_bcnt_ops_per_s"] / 1e12,
                "nominal_lds_GBps": LDS_PEAK / 1e9, "nominal_valu_Tops": VALU_PEAK / 1e12}
    roof_valu["peak_measured"] = ceil["valu_int32_ops_per_s"] / 1e12
    roof_valu["frac_measured"] = valu_ach / ceil["valu_int32_ops_per_s"]
    roof_lds["peak_measured"] = lds_peak / 1e9
    roof_lds["frac_measured"] = lds_ach / lds_peak
    log("ceilings: %s; phases: %s" % (ceilings, sieve_phase))

    cpu = None
    if not args.no_cpu_baseline:
        nthreads = min(16, os.cpu_count() or 1)
        log("cpu baseline (oracle, %d threads, ~%.0f s)" % (nthreads, args.cpu_seconds))
        cpu = cpu_baseline(lo, hi, args.cpu_seconds, nthreads)

    log("per-n mode: %d bytes per call" % n_odd)
    per_n = bench_per_n(lo, hi, n_odd, ref)
    per_n["roofline"]["traffic"] = traffic.get("per_n")
    log("sieve alone: %d bits per call" % n_odd)
    sieve = bench_sieve(lo, hi)
    sieve["roofline"]["traffic"] = traffic.get("sieve")

    extras = {}
    if not args.no_extras:
        log("batched: 4096 intervals")
        extras["batched"] = bench_batched(steps=5)
        log("served: Poisson stream, 11 s")
        extras["served"] = bench_served()

    r0 = res[0]
    out = {
        "metric": "odd n verified/sec near 2^50 (1 GPU)",
        "value": value,
        "unit": "odd n/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": n_warm,
        "ms_per_step": elapsed / args.steps * 1e3,
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
            "streams": len(streams),
        },
        "roofline": roof,
        "roofline_alt": alt,
        "cpu_baseline": cpu,
        "latency_p50_ms": extras.get("served", {}).get("p50_ms"),
        "latency_p99_ms": extras.get("served", {}).get("p99_ms"),
        "ceilings": ceilings,
        "sieve_phase": sieve_phase,
        "per_n": per_n,
        "sieve": sieve,
        "batched": extras.get("batched"),
        "served": extras.get("served"),
        "result": {"kmax_seen": r0["kmax_seen"], "ksum": r0["ksum"],
                   "records": r0["records"], "n_exceptions": r0["n_exceptions"]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
