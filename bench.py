#!/usr/bin/env python3
"""Benchmark of the discord-search hot path on one MI355X.

One step = one complete exact discord search through the C ABI on a series
already resident in HBM: discord_prepare (eq. (2) statistics, PAA/SAX words,
Cand, Index_Word, row statistics) + discord_search (the pair-distance scan with
early abandon, row minima, device argmax, FP64 certification).  The workload is
the m = 2^20 random walk with four planted anomalies and window n = 128,
searched with the plain FP32 scan and exact early abandon.

Printed: one JSON line.  `value` is the time to discord in ms (prepare +
search + FP64 certification, series already in HBM; lower is better).  Beside
it: the brute-force-equivalent rate P(N, n) / time, the split-BF16
MFMA search of the same input (`mixed`), the time to discord under each
visiting order, full-scan rates of both precisions, the roofline of each scan
kernel (kernel time from HIP events on the plan's stream), the m = 2^20, n = 256
noisy walk in both precisions, per-window z-normalisation, time to discord
against the number of compute units (CU-limited streams), the 10^7-point walk
at windows of 1024 and 2048, the serving stream (p50/p99 latency and throughput,
at its 200 req/s and replayed 8x faster to saturate the server) and the FP64
CPU oracle: the whole m = 4096 case in full, and a bounded sample of rows of
the main workload, on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
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

# The paper's own numbers (Xeon Phi 7290 KNL, 288 threads, real SCD series):
# context only, another machine and another dataset.
PAPER_CONTEXT = {
    "phidd_knl7290_288thr_scd1m_n128_s": 10.4,
    "phidd_knl7290_288thr_scd10m_n128_s": 81.9,
    "phidd_knl7290_10thr_scd1m_n128_s": 109.2,
    "hotsax_corei5_scd1m_n128_s": 147600.0,
}

SCAN_SOURCES = {"k_scan_fp32": "scan_fp32.hip", "k_scan_mfma": "scan_mfma.hip"}


def scan_kernel(n: int, precision: str) -> str:
    """The scan kernel a search of window n runs in this precision."""
    return "k_scan_fp32" if precision == "fp32" else "k_scan_mfma"


def pair_count(N: int, n: int) -> int:
    return (N - n) * (N - n + 1) if N > n else 0


def scan_flops_per_pair(n: int, precision: str) -> float:
    # FP32 direct form: per term one subtract, one multiply, one add.
    # split-BF16: three n-long bf16 dot products, 2 flop per term each.
    return 3.0 * n if precision == "fp32" else 6.0 * n


def source_sha(kernel: str) -> str:
    p = os.path.join(ROOT, "paper_1901_00155_amd", "csrc", SCAN_SOURCES[kernel])
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def traffic_for(precision: str, workload: str, mode: str, n: int):
    """HBM bytes of the scan launches of one search, from the committed
    rocprofv3 PMC summary, if it was taken on the current kernel source; else
    None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(p))[f"{precision}/{workload}/{mode}"]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("source_sha") != source_sha(scan_kernel(n, precision)):
        return None
    return rec.get("bytes_per_search")


def time_steps(dd, Td, n, precision, abandon, steps, warmup, order=2, znorm=False,
               per_step=None, plan=False):
    """Mean seconds per step over `steps` timed steps after `warmup` untimed
    ones, and the steps' results.  A step is one discord_search_once call
    (preparation and search as one device sequence, one synchronisation), or
    with `plan` discord_prepare + discord_search on a new plan (a
    synchronisation after each).  Each step returns once its result is on the
    host, so `per_step` (a list, if given) receives every timed step's own
    duration in ms as well."""
    import torch
    results = []
    stream = torch.cuda.current_stream()
    t_prev = 0.0
    for it in range(warmup + steps):
        if it == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t_prev = t0
        if plan:
            with dd.Plan(Td, n, precision=precision, abandon=abandon, order=order, stream=stream,
                         torch_workspace=True, znorm=znorm) as p:
                r = p.search()
        else:
            r = dd.search_once(Td, n, precision=precision, abandon=abandon, order=order,
                               stream=stream, znorm=znorm)
        if it >= warmup:
            results.append(r)
            if per_step is not None:
                t_now = time.perf_counter()
                per_step.append((t_now - t_prev) * 1e3)
                t_prev = t_now
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) / max(steps, 1), results


def roofline(n, precision, pairs, scan_ms, traffic, launches=None):
    """Algorithmic flops of the scan launches (pairs x flops per pair) over
    their summed HIP-event time, against the chip's peak.  Averaged over the
    launches of a search, this is the per-launch figure (total work / total
    time).  traffic: HBM bytes per search from the committed PMC summary, with
    the launch count it covers, or None."""
    flops = scan_flops_per_pair(n, precision) * pairs
    achieved = flops / (scan_ms * 1e-3) / 1e12
    peak = PEAK_FP32_VECTOR_TFLOPS if precision == "fp32" else PEAK_BF16_MFMA_TFLOPS
    return {"bound": "alu" if precision == "fp32" else "mfma", "achieved": achieved,
            "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
            "kernel": scan_kernel(n, precision),
            "flops_per_pair": scan_flops_per_pair(n, precision), "scan_ms": scan_ms,
            "launches": launches}


def cpu_config1(dd, workloads):
    """The m = 4096, n = 64 case (one series, planted sine) in full: the FP64
    oracle's brute force on the host cores against the GPU's time to discord."""
    import oracle
    import torch
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    w = workloads.small()
    t = time.perf_counter()
    ref = oracle.discord(w.series, w.n, threads=threads)
    dt = time.perf_counter() - t
    Td = torch.from_numpy(w.series).cuda()
    sec, res = time_steps(dd, Td, w.n, "fp32", True, 10, 3)
    r = res[-1]
    assert int(r.index) == ref["index"] and r.nn_index == ref["nn_index"]
    P = pair_count(w.m - w.n + 1, w.n)
    return {"workload": f"{w.name}: m={w.m} random walk, sine planted at [2000, 2064), n={w.n}",
            "oracle_s": dt, "oracle_pairs_per_s": P / dt, "cores": threads,
            "gpu_time_to_discord_ms": sec * 1e3, "index": int(r.index),
            "distance": float(r.distance), "oracle_distance": ref["distance"]}


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


def serving(dd, workloads, precision="bf16x3", slots=4, budget=8 << 30, count=4096, speed=1.0,
            reqs=None, label=None):
    """A request stream (by default the serving configuration's: Poisson
    arrivals at 200 req/s, m log-uniform in [2^12, 2^18], n in {64, 128, 256},
    one planted anomaly each) replayed open-loop through the serving loop, at
    its own rate (speed 1) or compressed in time (speed > 1) to saturate the
    server."""
    from paper_1901_00155_amd import serve
    t = time.perf_counter()
    if reqs is None:
        reqs = workloads.serve_requests(count=count)
    gen_s = time.perf_counter() - t
    with dd.Server(budget, slots=slots, precision=precision) as s:
        for r in reqs[:8]:                     # warm the slots' streams and staging
            s.submit(r.series, r.n, 10 ** 9 + r.tag)
        got = 0
        while got < 8:
            got += len(s.poll(64, 100))
        out = serve.replay(s, reqs, speed=speed, timeout_s=600)
    sm = out["summary"]
    recs = list(out["records"].values())
    ok = [c for c in recs if c["status"] == 0]
    assert sm["failed"] == 0 and all(c["result"]["certified"] == 1 for c in ok)
    modes = [c["result"]["graph"] for c in ok]
    return {
        "workload": label or (f"{count} requests, Poisson 200 req/s, m log-uniform [2^12, 2^18], "
                              "n in {64,128,256}, random walk + 1 planted anomaly each (seed 4)"),
        # how each completed request was launched: ordinary launches, captured
        # into a HIP graph, or a replay of its slot's graph
        "launch_modes": {"ordinary": modes.count(0), "captured": modes.count(1),
                         "graph_replay": modes.count(2)},
        "speed": speed, "precision": precision, "slots": slots, "hbm_budget_bytes": budget,
        "p50_ms": sm["p50_ms"], "p99_ms": sm["p99_ms"], "mean_ms": sm["mean_ms"],
        "max_ms": sm["max_ms"], "throughput_rps": sm["throughput_rps"],
        "offered_rps": sm["offered_rps"], "completed": sm["completed_ok"],
        "failed": sm["failed"], "rejected": sm["rejected"],
        "queue_p99_ms": sm["queue_p99_ms"], "service_p50_ms": sm["service_p50_ms"],
        "service_p99_ms": sm["service_p99_ms"], "mean_concurrency": sm["mean_concurrency"],
        "peak_running": sm["peak_running"], "peak_bytes_in_use": sm["peak_bytes_in_use"],
        "pairs_evaluated_total": float(sum(c["result"]["pairs_evaluated"] for c in ok)),
        "span_s": sm["span_s"], "generate_s": gen_s,
    }


def noisy_block(dd, workloads):
    """The mixed-precision configuration: m = 2^20 walk + N(0, 0.05), n = 256;
    time to discord and full-scan rates of both precisions on the same input."""
    import torch
    w = workloads.noisy1m()
    Td = torch.from_numpy(w.series).cuda()
    N = w.m - w.n + 1
    blk = {"workload": f"{w.name}: m={w.m} walk + N(0, 0.05) noise, window n={w.n}",
           "brute_force_pairs": pair_count(N, w.n)}
    ref = None
    for prec in ("fp32", "bf16x3"):
        so, ro = time_steps(dd, Td, w.n, prec, True, 3, 1)
        y = ro[-1]
        ref = ref or (int(y.index), y.d2)
        assert (int(y.index), y.d2) == ref, "precisions disagree on noisy1m"
        _, rf = time_steps(dd, Td, w.n, prec, False, 1, 0)
        f = rf[-1]
        assert int(f.index) == ref[0]
        blk[prec] = {"time_to_discord_ms": so * 1e3, "index": int(y.index),
                     "distance": float(y.distance),
                     "max_rel_err_of_approx_nn": float(y.max_rel_err),
                     "full_scan_ms": f.ms_scan,
                     "full_scan_pairs_per_s": f.pairs_evaluated / (f.ms_scan * 1e-3),
                     "full_scan_roofline_frac": roofline(w.n, prec, f.pairs_evaluated, f.ms_scan,
                                                         None)["frac"]}
        print(f"# noisy1m {prec}: {so * 1e3:.1f} ms to discord, full scan {f.ms_scan:.1f} ms",
              file=sys.stderr, flush=True)
    blk["bf16x3_full_scan_speedup_vs_fp32"] = (blk["fp32"]["full_scan_ms"]
                                               / blk["bf16x3"]["full_scan_ms"])
    blk["bf16x3_time_to_discord_speedup_vs_fp32"] = (blk["fp32"]["time_to_discord_ms"]
                                                     / blk["bf16x3"]["time_to_discord_ms"])
    return blk


def znorm_block(dd, Td, w):
    """Per-window z-normalisation (each window normalised on its own) on the
    main workload: time to discord in both precisions."""
    blk = {"workload": f"{w.name}, every window z-normalised on its own"}
    ref = None
    for prec in ("fp32", "bf16x3"):
        so, ro = time_steps(dd, Td, w.n, prec, True, 3, 1, znorm=True)
        y = ro[-1]
        ref = ref or (int(y.index), y.d2)
        assert (int(y.index), y.d2) == ref, "precisions disagree under znorm"
        blk[prec] = {"time_to_discord_ms": so * 1e3, "index": int(y.index),
                     "distance": float(y.distance), "pairs_evaluated": float(y.pairs_evaluated),
                     "max_rel_err_of_approx_nn": float(y.max_rel_err)}
        print(f"# znorm {prec}: {so * 1e3:.1f} ms", file=sys.stderr, flush=True)
    return blk


def long_window_block(dd, workloads, windows=(1024, 2048)):
    """The paper's larger series and longer windows: a 10^7-point walk with
    eight planted anomalies, time to discord per window (split-BF16 where the
    window is within its limit, FP32 always)."""
    import torch
    blk = {}
    for n in windows:
        w = workloads.walk10m(n)
        Td = torch.from_numpy(w.series).cuda()
        row = {"m": w.m, "n": n, "brute_force_pairs": pair_count(w.m - n + 1, n)}
        ref = None
        for prec in ("fp32", "bf16x3"):
            if prec == "bf16x3" and n > dd.MIXED_MAX_N:
                continue
            so, ro = time_steps(dd, Td, n, prec, True, 1, 0)   # library already warm
            y = ro[-1]
            ref = ref or (int(y.index), y.d2)
            assert (int(y.index), y.d2) == ref, "precisions disagree on walk10m"
            row[prec] = {"time_to_discord_ms": so * 1e3, "index": int(y.index),
                         "distance": float(y.distance),
                         "pairs_evaluated": float(y.pairs_evaluated)}
            print(f"# walk10m n={n} {prec}: {so * 1e3:.1f} ms", file=sys.stderr, flush=True)
        blk[w.name] = row
        del Td
    return blk


def scalability_block(dd, Td, w, cu_counts=(8, 16, 32, 64, 128, 256)):
    """Time to discord against the number of compute units the search may use
    (CU-limited streams), the GPU form of the paper's scalability study:
    speedup s(k) = T(k0) / T(k) and efficiency e(k) = s(k) k0 / k from the
    smallest count k0 (one CU per die of the device at k0 = 8)."""
    blk = {"workload": w.name, "cu_counts": list(cu_counts), "base_cus": cu_counts[0]}
    for prec in ("fp32", "bf16x3"):
        rows = []
        for k in cu_counts:
            with dd.CULimitedStream(k) as cs:
                ts = []
                for it in range(3):
                    t = time.perf_counter()
                    r = dd.search_once(Td, w.n, precision=prec, stream=cs)
                    ts.append(time.perf_counter() - t)
            rows.append({"cus": k, "time_to_discord_ms": min(ts[1:]) * 1e3, "index": int(r.index),
                         "pairs_evaluated": float(r.pairs_evaluated)})
            print(f"# scalability {prec} {k} CUs: {rows[-1]['time_to_discord_ms']:.1f} ms",
                  file=sys.stderr, flush=True)
        t0 = rows[0]["time_to_discord_ms"]
        for row in rows:
            row["speedup"] = t0 / row["time_to_discord_ms"]
            row["efficiency"] = row["speedup"] * cu_counts[0] / row["cus"]
        assert len({row["index"] for row in rows}) == 1, "CU counts disagree"
        blk[prec] = rows
    return blk


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="walk1m")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--no-abandon", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--order", type=int, default=2, choices=[0, 1, 2])
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
    mode = "abandon" if abandon else "full"

    print(f"# workload {w.name}: m={m} n={n} N={N} P={P:.4e}", file=sys.stderr, flush=True)
    step_ms = []
    sec, res = time_steps(dd, Td, n, args.precision, abandon, args.steps, args.warmup, args.order,
                          per_step=step_ms)
    r = res[-1]
    assert len({int(x.index) for x in res}) == 1, "steps disagree"
    pairs = float(np.mean([x.pairs_evaluated for x in res]))
    scan_ms = float(np.mean([x.ms_scan for x in res]))
    print(f"# {args.precision} step {sec * 1e3:.2f} ms, scan {scan_ms:.2f} ms, index {r.index} "
          f"d={r.distance:.6f}", file=sys.stderr, flush=True)

    out = {
        "metric": "subseq-pair distances/s & time-to-discord vs plain FP32; serve p50/p99 ms",
        "value": sec * 1e3,
        "unit": "ms (time to discord)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16x3",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: m={m} seeded series, {len(w.anomalies)} planted "
                               f"anomalies, window n={n}", "m": m, "n": n,
                   "precision": args.precision, "abandon": abandon,
                   "order": {0: "matrix", 1: "phidd", 2: "cand+near-first"}[args.order]},
        "time_to_discord_ms": sec * 1e3,
        "time_to_discord_median_ms": float(np.median(step_ms)),
        "time_to_discord_p90_ms": float(np.percentile(step_ms, 90)),
        "brute_force_equiv_pairs_per_s": P / sec,
        "pairs_evaluated": pairs,
        "discord": {"index": int(r.index), "nn_index": int(r.nn_index),
                    "distance": float(r.distance), "d2": float(r.d2),
                    "certified": int(r.certified), "rows_rescored": int(r.rows_rescored),
                    "rows_abandoned": int(r.rows_abandoned),
                    "max_rel_err_of_approx_nn": float(r.max_rel_err)},
        "roofline": roofline(n, args.precision, pairs, scan_ms,
                             traffic_for(args.precision, w.name, mode, n),
                             launches=int(np.mean([x.scan_launches for x in res]))),
        "paper_context": PAPER_CONTEXT,
    }
    if not args.no_extras:
        # the same step from the host series: the 4 MB host-to-device copy of T
        # (and the readback, in every step anyway) inside the timed region
        hs = {}
        for prec in ("fp32", "bf16x3"):
            hms = []
            sh, _ = time_steps(dd, w.series, n, prec, abandon, max(args.steps, 5), args.warmup,
                               args.order, per_step=hms)
            hs[prec] = {"time_to_discord_ms": sh * 1e3,
                        "time_to_discord_median_ms": float(np.median(hms))}
        out["host_series"] = hs
        # the same step as discord_prepare + discord_search on a new plan: one
        # synchronisation after the preparation and one after the search
        pp = {}
        for prec in ("fp32", "bf16x3"):
            sp, _ = time_steps(dd, Td, n, prec, abandon, args.steps, args.warmup, args.order,
                               plan=True)
            pp[prec] = {"time_to_discord_ms": sp * 1e3}
        out["plan_path"] = pp
        print(f"# plan path: fp32 {pp['fp32']['time_to_discord_ms']:.2f} ms, "
              f"bf16x3 {pp['bf16x3']['time_to_discord_ms']:.2f} ms", file=sys.stderr, flush=True)
        print(f"# host series: fp32 {hs['fp32']['time_to_discord_ms']:.2f} ms, "
              f"bf16x3 {hs['bf16x3']['time_to_discord_ms']:.2f} ms", file=sys.stderr, flush=True)
        other = "bf16x3" if args.precision == "fp32" else "fp32"
        s2, rr = time_steps(dd, Td, n, other, abandon, args.steps, args.warmup, args.order)
        x = rr[-1]
        assert int(x.index) == int(r.index) and x.d2 == r.d2, "precisions disagree"
        p2 = float(np.mean([y.pairs_evaluated for y in rr]))
        sm2 = float(np.mean([y.ms_scan for y in rr]))
        out["mixed" if other == "bf16x3" else "plain_fp32"] = {
            "precision": other, "time_to_discord_ms": s2 * 1e3, "pairs_per_s": p2 / s2,
            "brute_force_equiv_pairs_per_s": P / s2, "speedup_vs_step": sec / s2,
            "max_rel_err_of_approx_nn": float(x.max_rel_err),
            "roofline": roofline(n, other, p2, sm2, traffic_for(other, w.name, mode, n),
                                 launches=int(np.mean([y.scan_launches for y in rr])))}
        print(f"# {other} step {s2 * 1e3:.2f} ms", file=sys.stderr, flush=True)
        if abandon:
            # the paper's visiting order (PhiDD: Cand first, same-word columns first)
            # and plain matrix order, both precisions, for comparison
            orders = {}
            for oname, oval in (("phidd", 1), ("matrix", 0), ("cand+near-first", 2)):
                orders[oname] = {}
                for prec in ("fp32", "bf16x3"):
                    so, ro = time_steps(dd, Td, n, prec, True, 2, 1, oval)
                    assert int(ro[-1].index) == int(r.index) and ro[-1].d2 == r.d2
                    orders[oname][prec] = {
                        "time_to_discord_ms": so * 1e3,
                        "pairs_evaluated": float(np.mean([y.pairs_evaluated for y in ro]))}
                    print(f"# order {oname} {prec}: {so * 1e3:.1f} ms", file=sys.stderr,
                          flush=True)
            out["time_to_discord_by_order"] = orders
            # the large single instance: m = 2^22, n = 512, split-BF16 matrix resident
            wl = workloads.large4m()
            Tl = torch.from_numpy(wl.series).cuda()
            Pl = pair_count(wl.m - wl.n + 1, wl.n)
            large = {"workload": f"{wl.name}: m={wl.m} sinusoids + walk + noise, "
                                 f"{len(wl.anomalies)} planted anomalies, window n={wl.n}",
                     "brute_force_pairs": Pl}
            ref_l = None
            for prec in ("bf16x3", "fp32"):
                sl, rl = time_steps(dd, Tl, wl.n, prec, True, 2, 1, args.order)
                y = rl[-1]
                if ref_l is None:
                    ref_l = (int(y.index), y.d2)
                assert (int(y.index), y.d2) == ref_l, "precisions disagree on the large instance"
                large[prec] = {"time_to_discord_ms": sl * 1e3, "pairs_evaluated": float(y.pairs_evaluated),
                               "brute_force_equiv_pairs_per_s": Pl / sl,
                               "index": int(y.index), "distance": float(y.distance)}
                print(f"# large {prec}: {sl * 1e3:.1f} ms", file=sys.stderr, flush=True)
            out["large_instance"] = large
            del Tl
        full = {}
        for prec in ("fp32", "bf16x3"):
            _, rf = time_steps(dd, Td, n, prec, False, 1, 0)
            y = rf[-1]
            assert int(y.index) == int(r.index)
            full[prec] = {"pairs_per_s": y.pairs_evaluated / (y.ms_scan * 1e-3),
                          "scan_ms": y.ms_scan,
                          "roofline_frac": roofline(n, prec, y.pairs_evaluated, y.ms_scan,
                                                    None)["frac"]}
            print(f"# full scan {prec}: {y.ms_scan:.1f} ms", file=sys.stderr, flush=True)
        full["bf16x3_speedup_vs_fp32"] = full["fp32"]["scan_ms"] / full["bf16x3"]["scan_ms"]
        out["full_scan"] = full
        out["noisy1m"] = noisy_block(dd, workloads)
        if abandon:
            out["znorm"] = znorm_block(dd, Td, w)
            out["scalability"] = scalability_block(dd, Td, w)
            out["long_windows"] = long_window_block(dd, workloads)
    if not args.no_serve:
        reqs = workloads.serve_requests(count=4096)
        # one shape (a monitor re-searching a fixed-length window of a stream):
        # every slot replays its captured graph after two requests
        fixed = workloads.serve_requests(seed=6, count=2048, log2_min=14, log2_max=14,
                                         windows=(128,))
        fixed_label = ("2048 requests, Poisson 200 req/s, m = 2^14, n = 128, random walk + 1 "
                       "planted anomaly each (seed 6)")
        for key, speed, rq, label in (("serving", 1.0, reqs, None),
                                      ("serving_saturated", 8.0, reqs, None),
                                      ("serving_fixed_shape", 8.0, fixed, fixed_label)):
            out[key] = serving(dd, workloads, speed=speed, reqs=rq, label=label,
                               count=len(rq))
            sv = out[key]
            print(f"# {key} (x{speed:g}): p50 {sv['p50_ms']:.2f} ms p99 {sv['p99_ms']:.2f} ms "
                  f"{sv['throughput_rps']:.1f} req/s, mean concurrency {sv['mean_concurrency']:.2f}, "
                  f"launches {sv['launch_modes']}", file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w.series, n, args.cpu_budget)
        out["cpu_baseline"]["config1_full"] = cpu_config1(dd, workloads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
