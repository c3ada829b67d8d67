#!/usr/bin/env python3
"""Benchmark of the discord-search hot path on one MI355X.

One step = one complete exact discord search through the C ABI on a series
already resident in HBM: discord_prepare (eq. (2) statistics, PAA/SAX words,
Cand, Index_Word) + discord_search (the two-phase pair-distance scan with early
abandon, row minima, device argmax, FP64 certification).  The workload is the
m = 2^20 random walk with four planted anomalies and window n = 128.

Printed: one JSON line.  `value` is pair distances computed per second of step
time (the scan's own count of evaluated non-self pairs).  Extra fields give the
time to discord, the brute-force-equivalent rate P(N, n) / time, full-scan
rates of each precision, the roofline of the dominant kernel (the pair scan;
kernel time from HIP events on the plan's stream) and the FP64 CPU oracle timed
on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0


def pair_count(N: int, n: int) -> int:
    return (N - n) * (N - n + 1) if N > n else 0


def scan_flops_per_pair(n: int, precision: str) -> float:
    # direct form: per term one subtract, one multiply, one add
    if precision == "fp32":
        return 3.0 * n
    # split-BF16: three n-long dot products of 2 flops per term
    return 6.0 * n


def time_steps(dd, Td, n, precision, abandon, steps, warmup, ws_holder):
    import torch
    results = []
    stream = torch.cuda.current_stream()
    for it in range(warmup + steps):
        if it == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        with dd.Plan(Td, n, precision=precision, abandon=abandon, stream=stream,
                     torch_workspace=True) as p:
            r = p.search()
        if it >= warmup:
            results.append(r)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) / max(steps, 1), results


def cpu_baseline(series, n, budget_s=15.0):
    """FP64 oracle (plain C, OpenMP over rows) on a bounded sample of rows of the
    same workload: each sampled row against all N columns."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    N = series.size - n + 1
    rng = np.random.default_rng(12345)
    rows = rng.choice(N, size=min(N, 4 * threads), replace=False).astype(np.int64)
    t = time.perf_counter()
    oracle.rows_nn(series, n, rows, threads=threads)
    dt = time.perf_counter() - t
    per_row = dt / rows.size
    count = int(min(N, max(rows.size, budget_s / max(per_row, 1e-9))))
    count = (count + threads - 1) // threads * threads
    rows = rng.choice(N, size=min(N, count), replace=False).astype(np.int64)
    t = time.perf_counter()
    oracle.rows_nn(series, n, rows, threads=threads)
    dt = time.perf_counter() - t
    pairs = sum(int(N - max(0, min(N, i + n) - max(0, i - n + 1))) for i in rows)
    return {"value": pairs / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"exact FP64 NN of {rows.size} random rows x all {N} columns "
                      f"({pairs:.3e} pairs, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="walk1m")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--no-abandon", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1901_00155_amd as dd
    from paper_1901_00155_amd import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dd.load()
    w = workloads.by_name(args.workload)
    n, m = w.n, w.m
    N = m - n + 1
    P = pair_count(N, n)
    Td = torch.from_numpy(w.series).cuda()
    abandon = not args.no_abandon

    print(f"# workload {w.name}: m={m} n={n} N={N} P={P:.4e}", file=sys.stderr, flush=True)
    sec, res = time_steps(dd, Td, n, args.precision, abandon, args.steps, args.warmup, None)
    r = res[-1]
    idx = {int(x.index) for x in res}
    assert len(idx) == 1, "steps disagree"
    pairs = float(np.mean([x.pairs_evaluated for x in res]))
    scan_ms = float(np.mean([x.ms_scan for x in res]))
    print(f"# step {sec * 1e3:.2f} ms, scan {scan_ms:.2f} ms, index {r.index} "
          f"d={r.distance:.6f}", file=sys.stderr, flush=True)

    flops = scan_flops_per_pair(n, args.precision) * pairs
    achieved_tflops = flops / (scan_ms * 1e-3) / 1e12
    peak = PEAK_FP32_VECTOR_TFLOPS if args.precision == "fp32" else PEAK_BF16_MFMA_TFLOPS
    out = {
        "metric": "subseq-pair distances/s",
        "value": pairs / sec,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16x3",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: m={m} seeded series, {len(w.anomalies)} planted "
                               f"anomalies, window n={n}", "m": m, "n": n,
                   "precision": args.precision, "abandon": abandon, "order": "phidd"},
        "time_to_discord_ms": sec * 1e3,
        "brute_force_equiv_pairs_per_s": P / sec,
        "pairs_evaluated": pairs,
        "discord": {"index": int(r.index), "nn_index": int(r.nn_index),
                    "distance": float(r.distance), "certified": int(r.certified),
                    "rows_rescored": int(r.rows_rescored), "max_rel_err": float(r.max_rel_err)},
        "roofline": {"bound": "alu" if args.precision == "fp32" else "mfma",
                     "achieved": achieved_tflops, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved_tflops / peak, "traffic": None,
                     "kernel": "scan (pair-distance tiles)",
                     "flops_per_pair": scan_flops_per_pair(n, args.precision),
                     "scan_ms_per_launch": scan_ms},
    }
    if not args.no_extras:
        extras = {}
        for prec in ("fp32",):
            s2, rr = time_steps(dd, Td, n, prec, False, 1, 0, None)
            x = rr[-1]
            extras[prec] = {"full_scan_pairs_per_s": P / (x.ms_scan * 1e-3),
                            "step_ms": s2 * 1e3, "scan_ms": x.ms_scan, "index": int(x.index)}
            print(f"# full scan {prec}: {x.ms_scan:.1f} ms", file=sys.stderr, flush=True)
        out["full_scan"] = extras
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w.series, n, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
