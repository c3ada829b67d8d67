"""Open-loop replay of a request stream through the serving loop.

A submitter thread hands each request to ``Server.submit`` at its arrival time
(arrivals are fixed in advance, so a slow server does not slow the arrivals
down); the calling thread polls completions.  Latency is measured from the
request's scheduled arrival to the poll that returned its completion.
"""
from __future__ import annotations

import threading
import time

import numpy as np


def replay(server, requests, speed: float = 1.0, poll_ms: int = 2,
           timeout_s: float = 600.0) -> dict:
    """Replays `requests` (objects with arrival_s, series, n, tag) into `server`.

    Returns the summary (p50/p99/mean/max latency in ms over successful requests,
    throughput in requests/s over the span from the first arrival to the last
    completion, the server's counters) and the per-request records."""
    t0 = time.perf_counter() + 0.05
    arrival = {}
    submit_status = {}
    submit_done = threading.Event()

    def submitter():
        try:
            for r in requests:
                due = t0 + r.arrival_s / speed
                while True:
                    now = time.perf_counter()
                    if now >= due:
                        break
                    time.sleep(min(due - now, 0.002))
                arrival[r.tag] = due
                submit_status[r.tag] = server.submit(r.series, r.n, r.tag)
        finally:
            submit_done.set()

    th = threading.Thread(target=submitter, name="replay-submitter", daemon=True)
    th.start()
    records = {}
    deadline = time.perf_counter() + timeout_s
    while True:
        for c in server.poll(256, poll_ms):
            c["t_poll"] = time.perf_counter()
            records[c["tag"]] = c
        if submit_done.is_set():
            accepted = sum(1 for s in submit_status.values() if s == 0)
            if len(records) >= accepted:
                break
        if time.perf_counter() > deadline:
            raise TimeoutError(f"replay: {len(records)} of {len(requests)} requests completed "
                               f"within {timeout_s} s")
    th.join()
    stats = server.stats()
    lat = np.array([(c["t_poll"] - arrival[t]) * 1e3 for t, c in records.items()
                    if c["status"] == 0], dtype=np.float64)
    queue_ms = np.array([c["t_admit_ms"] - c["t_submit_ms"] for c in records.values()])
    service_ms = np.array([c["t_done_ms"] - c["t_admit_ms"] for c in records.values()])
    end = max([c["t_poll"] for c in records.values()], default=t0)
    span = max(end - t0, 1e-9)
    ok = int(lat.size)

    def pct(a, q):
        return float(np.percentile(a, q)) if a.size else None

    summary = {
        "requests": len(requests),
        "accepted": sum(1 for s in submit_status.values() if s == 0),
        "rejected": sum(1 for s in submit_status.values() if s != 0),
        "completed_ok": ok,
        "failed": sum(1 for c in records.values() if c["status"] != 0),
        "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "mean_ms": float(lat.mean()) if ok else None,
        "max_ms": float(lat.max()) if ok else None,
        "queue_p50_ms": pct(queue_ms, 50), "queue_p99_ms": pct(queue_ms, 99),
        "service_p50_ms": pct(service_ms, 50), "service_p99_ms": pct(service_ms, 99),
        "throughput_rps": ok / span,
        "offered_rps": len(requests) / max(requests[-1].arrival_s / speed, 1e-9) if requests else 0.0,
        "span_s": span,
        "mean_concurrency": stats["busy_ms"] / (span * 1e3),
        "peak_running": stats["peak_running"],
        "peak_bytes_in_use": stats["peak_bytes_in_use"],
        "budget_bytes": stats["budget_bytes"],
        "slots": stats["slots"],
    }
    return {"summary": summary, "records": records, "submit_status": submit_status}
