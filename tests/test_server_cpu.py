"""Host tests of the serving loop (discord_server_*) with fake executors: admission
by footprint, strict FIFO order, error isolation, submit-time refusals, shutdown
with queued work, the replay driver's latency accounting, and the scheduler under
ThreadSanitizer and AddressSanitizer.  No GPU: the scheduler is plain host code
and the executor is pluggable."""
import os
import shutil
import subprocess
import threading
import time

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.fixture(scope="module")
def dd():
    import paper_1901_00155_amd as dd
    if not os.path.exists(dd.LIB_PATH):
        pytest.fail("libdiscord.so is not built: run __graft_entry__.build()")
    dd.load()
    return dd


def _drain(server, count, timeout_s=30.0):
    out = []
    deadline = time.time() + timeout_s
    while len(out) < count:
        out += server.poll(64, 20)
        assert time.time() < deadline, f"only {len(out)} of {count} completions"
    return out


class LiveBlocks:
    """Executor that checks, while it runs, that the arena blocks of all running
    requests are disjoint and within the budget."""

    def __init__(self, budget, delay_s=0.01, result=None):
        self.budget, self.delay_s, self.result = budget, delay_s, result
        self.live = {}
        self.lock = threading.Lock()
        self.errors = []
        self.peak = 0
        self.calls = []

    def __call__(self, req, opts, res):
        with self.lock:
            off, b = req.ws_offset, req.ws_bytes
            for o2, b2 in self.live.values():
                if not (off + b <= o2 or o2 + b2 <= off):
                    self.errors.append(("overlap", req.tag))
            if sum(b2 for _, b2 in self.live.values()) + b > self.budget:
                self.errors.append(("budget", req.tag))
            if req.workspace is not None:
                self.errors.append(("virtual arena has a device pointer", req.tag))
            self.live[req.tag] = (off, b)
            self.peak = max(self.peak, len(self.live))
            self.calls.append(req.tag)
        time.sleep(self.delay_s)
        T = np.ctypeslib.as_array(req.T, shape=(req.m,))
        res.index = int(np.argmax(T))
        res.d2 = float(T.astype(np.float64).sum())
        with self.lock:
            del self.live[req.tag]
        return 0


def test_admission_by_footprint(dd):
    m, n = 8192, 64
    fp = dd.workspace_bytes(m, n)
    budget = int(2.5 * ((fp + 255) // 256 * 256))
    ex = LiveBlocks(budget, delay_s=0.02)
    with dd.Server(budget, slots=4, executor=ex) as s:
        rng = np.random.default_rng(0)
        for t in range(12):
            assert s.submit(rng.standard_normal(m).astype(np.float32), n, t) == 0
        done = _drain(s, 12)
        st = s.stats()
    assert not ex.errors, ex.errors
    assert ex.peak == 2                       # the budget, not the 4 slots, binds
    assert st["peak_running"] == 2 and st["peak_bytes_in_use"] <= budget
    assert st["bytes_in_use"] == 0 and st["running"] == 0 and st["queued"] == 0
    assert st["completed"] == 12 and st["failed"] == 0
    assert sorted(c["tag"] for c in done) == list(range(12))
    for c in done:
        assert c["t_submit_ms"] <= c["t_admit_ms"] <= c["t_done_ms"]
        assert c["ws_bytes"] == (fp + 255) // 256 * 256


def test_slots_bind_when_memory_is_plentiful(dd):
    ex = LiveBlocks(1 << 30, delay_s=0.02)
    with dd.Server(1 << 30, slots=3, executor=ex) as s:
        for t in range(9):
            assert s.submit(np.arange(4096, dtype=np.float32), 64, t) == 0
        _drain(s, 9)
        st = s.stats()
    assert ex.peak == 3 and st["peak_running"] == 3
    assert not ex.errors


def test_slot_keeps_its_block_for_one_shape(dd):
    """A slot serving requests of one footprint gets its previous arena block
    back (so a captured graph of the request keeps its device addresses), even
    where first-fit would hand it another free block."""
    m, n = 8192, 64
    fp = (dd.workspace_bytes(m, n) + 255) // 256 * 256
    seen = {}
    lock = threading.Lock()

    def ex(req, opts, res):
        with lock:
            seen.setdefault(req.slot, []).append(req.ws_offset)
        time.sleep(0.002 * (1 + req.slot))    # the slots drift apart
        res.index = 0
        return 0

    with dd.Server(4 * fp, slots=3, executor=ex) as s:
        for t in range(30):
            assert s.submit(np.arange(m, dtype=np.float32), n, t) == 0
        _drain(s, 30)
    assert sum(len(v) for v in seen.values()) == 30 and len(seen) == 3
    for slot, offs in seen.items():
        assert len(set(offs)) == 1, (slot, offs)
    assert len({offs[0] for offs in seen.values()}) == 3   # disjoint blocks


def test_strict_fifo_admission(dd):
    """A request at the head that does not fit yet is not overtaken by smaller
    ones behind it (no starvation); admission order equals submission order."""
    small_m, big_m, n = 4096, 65536, 64
    big = (dd.workspace_bytes(big_m, n) + 255) // 256 * 256
    small = (dd.workspace_bytes(small_m, n) + 255) // 256 * 256
    budget = big + small                       # the big one fits only alone with one small
    ex = LiveBlocks(budget, delay_s=0.01)
    with dd.Server(budget, slots=4, executor=ex) as s:
        sizes = [small_m, small_m, big_m, small_m, small_m, big_m, small_m]
        for t, m in enumerate(sizes):
            assert s.submit(np.ones(m, dtype=np.float32) + np.arange(m, dtype=np.float32), n, t) == 0
        done = _drain(s, len(sizes))
    assert not ex.errors
    order = [c["tag"] for c in sorted(done, key=lambda c: c["t_admit_ms"])]
    assert order == list(range(len(sizes)))


def test_failures_complete_with_status_and_do_not_poison(dd):
    def ex(req, opts, res):
        if req.tag == 3:
            return -2                          # e.g. a constant series
        if req.tag == 5:
            raise RuntimeError("executor blew up")
        res.index = req.tag
        return 0

    with dd.Server(1 << 28, slots=2, executor=ex) as s:
        for t in range(8):
            assert s.submit(np.arange(4096, dtype=np.float32), 64, t) == 0
        done = {c["tag"]: c for c in _drain(s, 8)}
        st = s.stats()
    assert done[3]["status"] == -2
    assert done[5]["status"] == -4 and "executor blew up" in done[5]["detail"]
    for t in (0, 1, 2, 4, 6, 7):
        assert done[t]["status"] == 0 and done[t]["result"]["index"] == t
    assert done[3]["result"]["index"] == 0     # no output written on failure
    assert st["failed"] == 2 and st["completed"] == 8 and st["bytes_in_use"] == 0


def test_submit_refusals(dd):
    release = threading.Event()

    def ex(req, opts, res):
        release.wait(10)
        return 0

    budget = 4 << 20
    with dd.Server(budget, slots=1, max_queued=2, executor=ex) as s:
        T = np.arange(8192, dtype=np.float32)
        assert s.submit(T[:100], 64, 0) == -1          # m < 2n
        assert s.submit(T, 0, 1) == -1                 # n < 1
        assert s.submit(np.arange(1 << 21, dtype=np.float32), 64, 2) == -3   # never fits
        assert s.submit(T, 64, 3) == 0                 # runs (blocks in the executor)
        deadline = time.time() + 10
        while s.stats()["running"] != 1:
            assert time.time() < deadline
            time.sleep(0.005)
        assert s.submit(T, 64, 4) == 0                 # queued
        assert s.submit(T, 64, 5) == 0                 # queued
        assert s.submit(T, 64, 6) == -5                # queue full
        release.set()
        done = _drain(s, 3)
        st = s.stats()
    assert sorted(c["tag"] for c in done) == [3, 4, 5]
    assert st["rejected"] == 4 and st["submitted"] == 3
    with dd.Server(1 << 30, slots=1, executor=lambda *a: 0, precision="bf16x3") as s:
        assert s.submit(np.arange(4200, dtype=np.float32), 2049, 0) == -6   # beyond the MFMA limit


def test_bad_config_is_refused(dd):
    with pytest.raises(dd.DiscordError):
        dd.Server(1 << 20, slots=0, executor=lambda *a: 0)
    with pytest.raises(dd.DiscordError):
        dd.Server(1 << 20, slots=65, executor=lambda *a: 0)
    with pytest.raises(dd.DiscordError):
        dd.Server(1 << 20, slots=1, executor=lambda *a: 0, paa_w=9)


def test_destroy_with_queued_requests_returns(dd):
    def ex(req, opts, res):
        time.sleep(0.01)
        return 0

    s = dd.Server(1 << 30, slots=2, executor=ex)
    for t in range(50):
        assert s.submit(np.arange(4096, dtype=np.float32), 64, t) == 0
    t0 = time.time()
    s.close()                                   # running ones finish, queued ones are dropped
    assert time.time() - t0 < 5.0


def test_results_depend_only_on_the_request(dd):
    """With a deterministic executor the result of each request is the same when
    it runs alone and when it runs among others (the scheduler shares no result
    state between requests)."""
    rng = np.random.default_rng(3)
    series = [rng.standard_normal(int(rng.integers(4096, 20000))).astype(np.float32)
              for _ in range(16)]

    def run(batch):
        ex = LiveBlocks(1 << 30, delay_s=0.001)
        with dd.Server(1 << 30, slots=4, executor=ex) as s:
            for t in batch:
                assert s.submit(series[t], 64, t) == 0
            return {c["tag"]: (c["result"]["index"], c["result"]["d2"]) for c in _drain(s, len(batch))}

    mix = run(list(range(16)))
    for t in (0, 7, 15):
        assert run([t])[t] == mix[t]


def test_replay_latency_accounting(dd):
    """Open-loop replay against a cost-model executor (service time proportional
    to m): every request completes, latency >= service time, p50 <= p99 <= max,
    and the throughput follows the offered rate when the server keeps up."""
    from paper_1901_00155_amd import serve, workloads
    reqs = workloads.serve_requests(seed=4, count=60, rate_hz=200.0, log2_min=12, log2_max=14)

    def ex(req, opts, res):
        time.sleep(req.m * 2e-7)               # 0.8 .. 3.3 ms
        return 0

    with dd.Server(1 << 30, slots=4, executor=ex) as s:
        out = serve.replay(s, reqs, speed=1.0, poll_ms=1, timeout_s=60)
    sm = out["summary"]
    assert sm["completed_ok"] == 60 and sm["rejected"] == 0 and sm["failed"] == 0
    assert sm["p50_ms"] <= sm["p99_ms"] <= sm["max_ms"]
    assert sm["p50_ms"] >= sm["service_p50_ms"] * 0.9
    assert 0.0 < sm["mean_concurrency"] <= 4.0
    assert 0.4 * sm["offered_rps"] < sm["throughput_rps"] < 1.6 * sm["offered_rps"]


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_scheduler_under_sanitizers(san, tmp_path):
    """tests/native/server_stress.cpp drives the scheduler from several submitter
    and poller threads with a fake executor; built with ThreadSanitizer or
    AddressSanitizer+UBSan (clang's runtimes, which intercept the clock-based
    condition-variable waits of libstdc++)."""
    if not os.path.exists(CLANG) and not shutil.which("clang++"):
        pytest.skip("clang++ not available")
    cxx = CLANG if os.path.exists(CLANG) else shutil.which("clang++")
    exe = str(tmp_path / "server_stress")
    subprocess.run([cxx, "-std=c++17", "-O1", "-g", f"-fsanitize={san}", "-fno-omit-frame-pointer",
                    os.path.join(ROOT, "tests", "native", "server_stress.cpp"),
                    os.path.join(ROOT, "paper_1901_00155_amd", "csrc", "server_core.cpp"),
                    "-o", exe, "-lpthread"], check=True, timeout=120)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66",
               ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "OK" in r.stdout and "WARNING" not in r.stderr


def test_replay_counts_failures_and_refusals(dd):
    """The replay summary separates refused submissions, failed completions and
    successful ones; latencies come only from successful requests."""
    from paper_1901_00155_amd import serve, workloads
    reqs = workloads.serve_requests(seed=9, count=30, rate_hz=500.0, log2_min=12, log2_max=13)
    reqs[4].n = 0                         # refused at submit (n < 1)

    def ex(req, opts, res):
        time.sleep(0.001)
        return -2 if req.tag % 7 == 3 else 0

    with dd.Server(1 << 30, slots=2, executor=ex) as s:
        out = serve.replay(s, reqs, timeout_s=60)
    sm = out["summary"]
    failing = sum(1 for r in reqs if r.tag % 7 == 3 and r.tag != 4)
    assert sm["rejected"] == 1 and out["submit_status"][4] == -1
    assert sm["failed"] == failing
    assert sm["completed_ok"] == len(reqs) - 1 - failing
    assert sm["p50_ms"] is not None and sm["p50_ms"] > 0
