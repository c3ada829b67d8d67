"""Seeded synthetic series for the discord-search workloads.

This module only draws random numbers and plants anomalies.  It holds none of
the discord method's arithmetic, so both the GPU path and the CPU oracle can
take their inputs from it.  Every series is generated in float64 with
``numpy.random.default_rng(seed)`` and cast to float32 once; the oracle and the
GPU then read the same float32 values.

The paper evaluates on two real series of 10^6 and 10^7 points (its dataset
table, section 4.1) that are not available here; the workloads below are
stand-ins with the same shape: long univariate series, windows of 64-2048
samples, and a few planted anomalous windows.

Workloads
---------
``small``     m=4096 random walk (seed 0), one sine anomaly over t[2000:2064], n=64.
``walk1m``    m=2^20 random walk (seed 1), n=128, four anomalies of 128 samples
              (sine, level shift, spike burst, sine) at seeded positions.
``noisy1m``   m=2^20 random walk plus N(0, 0.05) noise (seed 2), n=256, no anomaly.
``large4m``   m=2^22: three seeded sinusoids (periods 200-5000, log-uniform) plus a
              random walk plus N(0, 0.2) noise (seed 3), n=512, eight anomalies.
``walk10m``   m=10^7 random walk plus N(0, 0.1) noise (seed 5), eight anomalies
              cycling the three kinds, window n chosen by the caller (the
              paper's windows 64-2048 on its 10^7-point series).
``serve``     4096 requests (seed 4): Poisson arrivals at 200 req/s, lengths
              log-uniform in [2^12, 2^18], n uniform over {64, 128, 256}, one
              anomaly each.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ANOMALY_TYPES = ("sine", "level", "spikes")


@dataclasses.dataclass
class Workload:
    name: str
    series: np.ndarray          # float32[m]
    n: int
    anomalies: list             # [(position, length, kind)]
    seed: int

    @property
    def m(self) -> int:
        return int(self.series.shape[0])


def _plant(t: np.ndarray, rng: np.random.Generator, pos: int, n: int, kind: str) -> None:
    """Plant one anomaly of ``n`` samples at ``pos`` (in place, float64)."""
    k = np.arange(n, dtype=np.float64)
    if kind == "sine":
        t[pos:pos + n] = t[pos] + 10.0 * np.sin(2.0 * math.pi * k / n)
    elif kind == "level":
        t[pos:pos + n] += 20.0
    elif kind == "spikes":
        offs = rng.choice(n, size=8, replace=False)
        signs = rng.choice(np.array([-1.0, 1.0]), size=8)
        t[pos + offs] += 15.0 * signs
    else:
        raise ValueError(kind)


def _positions(rng: np.random.Generator, m: int, n: int, count: int) -> list:
    """Draw ``count`` anomaly starts in [2n, m-3n), pairwise at least 3n apart."""
    lo, hi = 2 * n, m - 3 * n
    if hi <= lo:
        raise ValueError("series too short for an anomaly")
    while True:
        pos = sorted(int(p) for p in rng.integers(lo, hi, size=count))
        if all(b - a >= 3 * n for a, b in zip(pos, pos[1:])):
            return pos


def small(seed: int = 0) -> Workload:
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.standard_normal(4096))
    k = np.arange(64, dtype=np.float64)
    t[2000:2064] = 3.0 * np.sin(2.0 * math.pi * k / 64) + rng.normal(0.0, 0.1, 64)
    return Workload("small", t.astype(np.float32), 64, [(2000, 64, "sine")], seed)


def walk1m(seed: int = 1, m: int = 1 << 20, n: int = 128) -> Workload:
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.standard_normal(m))
    kinds = ["sine", "level", "spikes", "sine"]
    pos = _positions(rng, m, n, len(kinds))
    for p, kind in zip(pos, kinds):
        _plant(t, rng, p, n, kind)
    return Workload("walk1m" if n == 128 else f"walk1m_n{n}", t.astype(np.float32), n,
                    [(p, n, kd) for p, kd in zip(pos, kinds)], seed)


def noisy1m(seed: int = 2, m: int = 1 << 20, n: int = 256) -> Workload:
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.standard_normal(m)) + rng.normal(0.0, 0.05, m)
    return Workload("noisy1m", t.astype(np.float32), n, [], seed)


def large4m(seed: int = 3, m: int = 1 << 22, n: int = 512) -> Workload:
    rng = np.random.default_rng(seed)
    periods = np.exp(rng.uniform(math.log(200.0), math.log(5000.0), 3))
    amps = rng.uniform(5.0, 20.0, 3)
    phases = rng.uniform(0.0, 2.0 * math.pi, 3)
    x = np.arange(m, dtype=np.float64)
    t = np.zeros(m)
    for P, A, ph in zip(periods, amps, phases):
        t += A * np.sin(2.0 * math.pi * x / P + ph)
    t += np.cumsum(rng.standard_normal(m)) + rng.normal(0.0, 0.2, m)
    kinds = [ANOMALY_TYPES[i % 3] for i in range(8)]
    pos = _positions(rng, m, n, len(kinds))
    for p, kind in zip(pos, kinds):
        _plant(t, rng, p, n, kind)
    return Workload("large4m", t.astype(np.float32), n,
                    [(p, n, kd) for p, kd in zip(pos, kinds)], seed)


def walk10m(n: int = 1024, seed: int = 5, m: int = 10 ** 7) -> Workload:
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.standard_normal(m)) + rng.normal(0.0, 0.1, m)
    kinds = [ANOMALY_TYPES[i % 3] for i in range(8)]
    pos = _positions(rng, m, n, len(kinds))
    for p, kind in zip(pos, kinds):
        _plant(t, rng, p, n, kind)
    return Workload(f"walk10m_n{n}", t.astype(np.float32), n,
                    [(p, n, kd) for p, kd in zip(pos, kinds)], seed)


@dataclasses.dataclass
class Request:
    arrival_s: float
    series: np.ndarray
    n: int
    anomaly: tuple
    tag: int


def serve_requests(seed: int = 4, count: int = 4096, rate_hz: float = 200.0,
                   log2_min: float = 12.0, log2_max: float = 18.0,
                   windows=(64, 128, 256)) -> list:
    """Open-loop request stream: Poisson arrivals, uneven (m, n), one anomaly each."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(count):
        m = int(math.floor(2.0 ** rng.uniform(log2_min, log2_max)))
        n = int(windows[int(rng.integers(0, len(windows)))])
        t = np.cumsum(rng.standard_normal(m))
        kind = ANOMALY_TYPES[r % 3]
        p = int(rng.integers(2 * n, m - 3 * n))
        _plant(t, rng, p, n, kind)
        out.append(Request(float(arrivals[r]), t.astype(np.float32), n, (p, n, kind), r))
    return out


def random_walk(m: int, seed: int, noise: float = 0.0) -> np.ndarray:
    """Plain seeded random walk (float32), for parity cases of arbitrary size."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.standard_normal(m))
    if noise:
        t = t + rng.normal(0.0, noise, m)
    return t.astype(np.float32)


def by_name(name: str) -> Workload:
    if name.startswith("walk10m"):           # walk10m or walk10m_n<window>
        return walk10m(int(name.split("_n")[1])) if "_n" in name else walk10m()
    if name.startswith("walk1m_n"):          # the 2^20 walk searched with another window
        return walk1m(n=int(name.split("_n")[1]))
    return {"small": small, "walk1m": walk1m, "noisy1m": noisy1m,
            "large4m": large4m}[name]()
