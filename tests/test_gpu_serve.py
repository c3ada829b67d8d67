"""GPU tests of the serving loop: every request's result is the same when it runs
alone (one plan, one stream) and when it runs in the mix with others overlapping
on the device, and equals the FP64 oracle where the oracle is quick; failing
requests complete with their status without disturbing the rest; an open-loop
replay completes every request with a certified result."""
import numpy as np
import pytest

import oracle
from paper_1901_00155_amd import workloads

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "bf16x3"]


def _requests(count=24, seed=4, log2_max=16):
    return workloads.serve_requests(seed=seed, count=count, rate_hz=200.0, log2_min=12,
                                    log2_max=log2_max)


def _drain(s, count, timeout_ms=120000):
    import time
    out = []
    t0 = time.time()
    while len(out) < count:
        out += s.poll(64, 100)
        assert (time.time() - t0) * 1e3 < timeout_ms, f"{len(out)} of {count} completed"
    return {c["tag"]: c for c in out}


@pytest.mark.parametrize("precision", PRECS)
def test_same_result_alone_and_in_the_mix(gpu, precision):
    dd = gpu
    reqs = _requests()
    alone = {}
    for r in reqs:
        with dd.Plan(r.series, r.n, precision=precision) as p:
            alone[r.tag] = p.search().as_dict()
    with dd.Server(4 << 30, slots=4, precision=precision) as s:
        for r in reqs:
            assert s.submit(r.series, r.n, r.tag) == 0
        mix = _drain(s, len(reqs))
        st = s.stats()
    assert st["peak_running"] >= 2, "requests did not overlap"
    assert st["failed"] == 0 and st["bytes_in_use"] == 0
    for r in reqs:
        c = mix[r.tag]
        assert c["status"] == 0, c["detail"]
        a, b = alone[r.tag], c["result"]
        assert b["certified"] == 1
        assert (b["index"], b["nn_index"]) == (a["index"], a["nn_index"]), r.tag
        assert b["d2"] == a["d2"] and b["distance"] == a["distance"], r.tag


@pytest.mark.parametrize("precision", PRECS)
def test_mix_matches_oracle_on_short_series(gpu, precision):
    dd = gpu
    reqs = [r for r in _requests(count=40, seed=7, log2_max=13)][:16]
    with dd.Server(2 << 30, slots=4, precision=precision) as s:
        for r in reqs:
            assert s.submit(r.series, r.n, r.tag) == 0
        mix = _drain(s, len(reqs))
    for r in reqs:
        ref = oracle.discord(r.series, r.n)
        got = mix[r.tag]["result"]
        assert mix[r.tag]["status"] == 0
        assert got["index"] == ref["index"], (r.tag, r.series.size, r.n)
        assert got["d2"] == pytest.approx(ref["d2"], rel=1e-9, abs=0)
        assert got["distance"] == pytest.approx(ref["distance"], rel=1e-9, abs=0)


@pytest.mark.parametrize("precision", PRECS)
def test_mix_certified_by_oracle_on_long_series(gpu, precision):
    """Served requests of 2^13 < m <= 2^18 samples, too long for the oracle's
    brute force: each result from the mix equals the same request run alone on
    a plan, and the witness array of that run is the oracle's FP64 certificate
    of the (index, d2) the server returned; the neighbour is the oracle's exact
    argmin of that row."""
    dd = gpu
    reqs = [r for r in workloads.serve_requests(seed=31, count=400, rate_hz=200.0, log2_min=12,
                                                log2_max=18) if r.series.size > 1 << 13][:16]
    assert len(reqs) == 16 and max(r.series.size for r in reqs) > 1 << 16
    with dd.Server(8 << 30, slots=4, precision=precision) as s:
        for r in reqs:
            assert s.submit(r.series, r.n, r.tag) == 0
        mix = _drain(s, len(reqs))
    for r in reqs:
        c = mix[r.tag]
        assert c["status"] == 0, c["detail"]
        got = c["result"]
        with dd.Plan(r.series, r.n, precision=precision) as p:
            a = p.search()
            wit = p.copy("nn_witness")
        assert (a.index, a.nn_index, a.d2) == (got["index"], got["nn_index"], got["d2"]), r.tag
        bad, first, nn = oracle.witness_check(r.series, r.n, got["index"], got["d2"], wit)
        assert bad == 0, (r.tag, first)
        assert got["d2"] == pytest.approx(nn, rel=1e-9, abs=0)
        d, j = oracle.rows_nn(r.series, r.n, [got["index"]])
        assert j[0] == got["nn_index"] and d[0] == nn


def test_failing_requests_do_not_disturb_the_mix(gpu):
    dd = gpu
    reqs = _requests(count=8, seed=11, log2_max=14)
    bad_const = np.full(8192, 3.0, dtype=np.float32)
    bad_nan = reqs[0].series.copy()
    bad_nan[100] = np.nan
    with dd.Server(2 << 30, slots=3, precision="bf16x3") as s:
        for r in reqs[:4]:
            assert s.submit(r.series, r.n, r.tag) == 0
        assert s.submit(bad_const, 64, 1000) == 0
        assert s.submit(bad_nan, reqs[0].n, 1001) == 0
        for r in reqs[4:]:
            assert s.submit(r.series, r.n, r.tag) == 0
        mix = _drain(s, len(reqs) + 2)
        st = s.stats()
    assert mix[1000]["status"] == -2 and mix[1001]["status"] == -1
    assert st["failed"] == 2 and st["bytes_in_use"] == 0
    for r in reqs:
        with dd.Plan(r.series, r.n, precision="bf16x3") as p:
            a = p.search()
        c = mix[r.tag]
        assert c["status"] == 0 and c["result"]["index"] == a.index and c["result"]["d2"] == a.d2


def test_open_loop_replay_completes(gpu):
    dd = gpu
    from paper_1901_00155_amd import serve
    reqs = workloads.serve_requests(seed=4, count=200, rate_hz=200.0)
    with dd.Server(8 << 30, slots=4, precision="bf16x3") as s:
        out = serve.replay(s, reqs, timeout_s=100)
    sm = out["summary"]
    assert sm["completed_ok"] == 200 and sm["failed"] == 0 and sm["rejected"] == 0
    assert all(c["result"]["certified"] == 1 for c in out["records"].values())
    assert sm["p50_ms"] <= sm["p99_ms"]
    print(sm)


def test_concurrent_submitters_many_slots(gpu):
    """Two host threads submit at once into a server with 8 slots (more streams
    than hardware queues); every result equals the request run alone."""
    import threading
    dd = gpu
    reqs = _requests(count=48, seed=21, log2_max=15)
    alone = {}
    for r in reqs:
        with dd.Plan(r.series, r.n, precision="bf16x3") as p:
            a = p.search()
            alone[r.tag] = (a.index, a.nn_index, a.d2)
    with dd.Server(4 << 30, slots=8, precision="bf16x3") as s:
        status = []

        def submit(part):
            for r in part:
                status.append(s.submit(r.series, r.n, r.tag))

        threads = [threading.Thread(target=submit, args=(reqs[k::2],)) for k in range(2)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        assert status.count(0) == len(reqs)
        mix = _drain(s, len(reqs))
        st = s.stats()
    assert st["peak_running"] >= 2 and st["failed"] == 0 and st["bytes_in_use"] == 0
    for r in reqs:
        c = mix[r.tag]
        assert c["status"] == 0, c["detail"]
        got = (c["result"]["index"], c["result"]["nn_index"], c["result"]["d2"])
        assert got == alone[r.tag], (r.tag, got, alone[r.tag])


@pytest.mark.parametrize("precision", PRECS)
def test_repeated_shape_replays_a_graph(gpu, precision):
    """Requests of one shape: on each slot the first runs with ordinary
    launches, the second is captured into a HIP graph and later ones replay it
    (result.graph 0, 1, 2).  Every result equals a plan's own search bit for
    bit, the first equals the FP64 oracle, and a failing request (NaN) in the
    stream neither breaks the replays after it nor changes their results."""
    dd = gpu
    m, n = 6000, 64
    series = [workloads.random_walk(m, seed=900 + k) for k in range(14)]
    bad = series[7].copy()
    bad[100] = np.nan
    series[7] = bad
    alone = {}
    for k, T in enumerate(series):
        if k == 7:
            continue
        with dd.Plan(T, n, precision=precision) as p:
            alone[k] = p.search().as_dict()
    o = oracle.discord(series[0], n)
    assert (alone[0]["index"], alone[0]["nn_index"]) == (o["index"], o["nn_index"])
    with dd.Server(1 << 30, slots=2, precision=precision) as s:
        for k, T in enumerate(series):
            assert s.submit(T, n, k) == 0
        done = _drain(s, len(series))
    assert done[7]["status"] == -1, done[7]["detail"]          # EINVAL: NaN in the series
    modes = [done[k]["result"]["graph"] for k in alone]
    print(precision, "graph modes", modes, flush=True)
    assert modes.count(2) >= 6 and modes.count(1) >= 1 and set(modes) <= {0, 1, 2}
    for k, a in alone.items():
        c = done[k]
        assert c["status"] == 0, c["detail"]
        b = c["result"]
        assert b["certified"] == 1
        assert (b["index"], b["nn_index"]) == (a["index"], a["nn_index"]), k
        assert b["d2"] == a["d2"] and b["distance"] == a["distance"], k


def test_plan_graph_reports_capture_then_replay(gpu):
    dd = gpu
    w = workloads.small()
    with dd.Plan(w.series, w.n) as p:
        r0 = p.search()
        r1 = p.search_graph()
        r2 = p.search_graph()
    assert (r0.graph, r1.graph, r2.graph) == (0, 1, 2)
    assert r0.index == r1.index == r2.index and r0.d2 == r1.d2 == r2.d2
