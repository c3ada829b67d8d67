"""Shared constructors of closed-form test series."""
import math

import numpy as np


def periodic_spike(rng, n):
    """Integer pattern of period P >= n tiled over >= 8 periods plus one spike h
    at p; returns (T, p, h) such that the closed form below holds."""
    while True:
        P = int(rng.integers(n, n + 6))
        pat = rng.integers(-20, 21, P).astype(np.int64)
        ext = np.concatenate([pat, pat, pat])
        dmin = min(int(((ext[a:a + n] - ext[b:b + n]) ** 2).sum())
                   for a in range(P) for b in range(P) if a != b) if P > 1 else 0
        h = int(math.floor(math.sqrt(dmin / 6.0)))
        if h >= 1 and 6 * h * h < dmin:
            break
    reps = int(rng.integers(8, 12))
    x = np.tile(pat, reps)
    p = int(rng.integers(2 * P, x.size - 2 * P))
    x[p] += h if rng.random() < 0.5 else -h
    return x.astype(np.float32), p, h
