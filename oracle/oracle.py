"""CPU oracle for discord search -- TEST INFRASTRUCTURE, not part of the product.

Plain FP64 implementations written from the paper (Polyakov & Zymbler, PhiDD):
the brute force of the definitions in section 2.1 (in C, see discord_ref.c),
and, in Python, independent companions used to pin it: a NumPy all-pairs brute
force, an exact-integer enumerator, Algorithm 1 (HOTSAX DiscordDiscovery) with
any visiting order, Algorithms 2-4 (PhiDD) and the SAX preparation structures of
section 3.1 (eqs. (3)-(10)).

Readings of the paper that this oracle takes (the paper is silent or garbled):
  * z-normalisation is global, eq. (2); it is affine, so the argmax is taken on
    raw-value squared distances and the distance is reported divided by sigma;
  * the lowest index wins ties in the argmax; the lowest j wins ties in the NN;
  * rows with no non-self match take no part in the argmax;
  * Algorithm 3's second inner loop updates ``min`` like Algorithm 4's does;
  * dist_bsf starts at 0 and pos_bsf at "none";
  * eq. (3) segments are [floor(s n / w), floor((s+1) n / w)); eq. (4) symbols are
    left-closed quantile intervals of N(0,1); eq. (9) is the lexicographic rank
    sum_s sym_s * |A|^(w-1-s) of the 0-based symbols.

A second reading is available everywhere as ``znorm=True``: Algorithm 2's
Znormalize(S) taken row by row, i.e. every window normalised by its own mean
and standard deviation (eq. (2) over the window), a flat window becoming the
zero vector.  Distances are then between normalised windows and are reported
as they are (no division by the series' sigma).
"""
from __future__ import annotations

import ctypes
import math
import os
import statistics

import numpy as np

__all__ = [
    "load", "stats", "pair_d2", "rows_nn", "discord", "witness_check", "sax_words",
    "np_sax_words", "breakpoints", "freq_cand", "index_word", "np_discord",
    "int_discord", "alg1", "phidd", "pair_count", "OracleError", "row_zstats",
    "np_discord_z", "exact_z_profile",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "lib", "liboracle.so")
_lib = None


class OracleError(ValueError):
    """Raised for inputs the definitions do not cover (status < 0)."""


def load():
    """Load the compiled C oracle, compiling it with gcc first if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    f64p = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    f32p = ctypes.POINTER(ctypes.c_float)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.orc_pair_d2.restype = ctypes.c_double
    lib.orc_pair_d2.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64]
    lib.orc_stats.restype = ctypes.c_int
    lib.orc_stats.argtypes = [f32p, ctypes.c_int64, f64p, f64p]
    lib.orc_rows_nn.restype = ctypes.c_int
    lib.orc_rows_nn.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, i64p, ctypes.c_int64,
                                f64p, i64p, ctypes.c_int]
    lib.orc_discord.restype = ctypes.c_int
    lib.orc_discord.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int,
                                i64p, i64p, f64p, f64p, f64p, f64p, i64p]
    lib.orc_witness_check.restype = ctypes.c_int64
    lib.orc_witness_check.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                      ctypes.c_double, i64p, ctypes.c_int, i64p, f64p]
    lib.orc_sax_words.restype = ctypes.c_int
    lib.orc_sax_words.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, f64p, ctypes.c_double, ctypes.c_double,
                                  i32p, ctypes.c_int]
    lib.orc_row_zstats.restype = ctypes.c_int
    lib.orc_row_zstats.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, f64p, f64p]
    lib.orc_pair_d2_z.restype = ctypes.c_double
    lib.orc_pair_d2_z.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_int64, f64p, f64p]
    lib.orc_rows_nn_z.restype = ctypes.c_int
    lib.orc_rows_nn_z.argtypes = lib.orc_rows_nn.argtypes
    lib.orc_discord_z.restype = ctypes.c_int
    lib.orc_discord_z.argtypes = lib.orc_discord.argtypes
    lib.orc_witness_check_z.restype = ctypes.c_int64
    lib.orc_witness_check_z.argtypes = lib.orc_witness_check.argtypes
    lib.orc_sax_words_z.restype = ctypes.c_int
    lib.orc_sax_words_z.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, f64p, f64p, f64p, i32p, ctypes.c_int]
    _lib = lib
    return lib


def _f32(T) -> np.ndarray:
    a = np.ascontiguousarray(T, dtype=np.float32)
    if a.ndim != 1:
        raise OracleError("series must be one-dimensional")
    return a


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _threads(threads):
    return int(threads) if threads else (os.cpu_count() or 1)


def pair_count(N: int, n: int) -> int:
    """Number of ordered pairs (i, j), 0 <= i, j < N, with |i - j| >= n."""
    if N - n <= 0:
        return 0
    return (N - n) * (N - n + 1)


def stats(T):
    """Mean and standard deviation of the series, eq. (2) (two-pass FP64)."""
    T = _f32(T)
    mu, sd = ctypes.c_double(), ctypes.c_double()
    st = load().orc_stats(_ptr(T, ctypes.c_float), T.size, ctypes.byref(mu), ctypes.byref(sd))
    if st == -2:
        raise OracleError("sigma == 0: eq. (2) is undefined for a constant series")
    if st != 0:
        raise OracleError("invalid series (empty or non-finite)")
    return mu.value, sd.value


def row_zstats(T, n: int):
    """Mean and standard deviation of every window T_{i,n} (eq. (2) over the
    window alone; two-pass, sequential sums in C).  Returns (mu[N], sigma[N])."""
    T = _f32(T)
    if n < 1 or T.size < n:
        raise OracleError("need 1 <= n <= m")
    N = T.size - n + 1
    mu = np.empty(N, dtype=np.float64)
    sg = np.empty(N, dtype=np.float64)
    load().orc_row_zstats(_ptr(T, ctypes.c_float), T.size, n, _ptr(mu, ctypes.c_double),
                          _ptr(sg, ctypes.c_double))
    return mu, sg


def pair_d2(T, n: int, i: int, j: int, znorm: bool = False) -> float:
    """Squared Euclidean distance of eq. (1) between T_{i,n} and T_{j,n} (with
    ``znorm``, between the two windows each normalised on its own)."""
    T = _f32(T)
    N = T.size - n + 1
    if not (0 <= i < N and 0 <= j < N):
        raise OracleError("row out of range")
    if znorm:
        mu, sg = row_zstats(T, n)
        return load().orc_pair_d2_z(_ptr(T, ctypes.c_float), T.size, n, i, j,
                                    _ptr(mu, ctypes.c_double), _ptr(sg, ctypes.c_double))
    return load().orc_pair_d2(_ptr(T, ctypes.c_float), T.size, n, i, j)


def rows_nn(T, n: int, rows, threads=None, znorm: bool = False):
    """Exact nearest non-self match (d^2, j) of each listed row; j = -1 if none."""
    T = _f32(T)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    N = T.size - n + 1
    if rows.size and (rows.min() < 0 or rows.max() >= N):
        raise OracleError("row out of range")
    d = np.empty(rows.size, dtype=np.float64)
    j = np.empty(rows.size, dtype=np.int64)
    fn = load().orc_rows_nn_z if znorm else load().orc_rows_nn
    st = fn(_ptr(T, ctypes.c_float), T.size, n, _ptr(rows, ctypes.c_int64),
                            rows.size, _ptr(d, ctypes.c_double), _ptr(j, ctypes.c_int64),
                            _threads(threads))
    if st != 0:
        raise OracleError("invalid arguments")
    return d, j


def discord(T, n: int, threads=None, profile: bool = False, znorm: bool = False) -> dict:
    """Brute-force discord of section 2.1 in FP64 (C).  Returns index, nn_index,
    d2 (raw squared NN distance), distance_raw, distance (z-normalised units,
    eq. (2)), mu, sigma and, if asked, the NN profile and its argmins.  With
    ``znorm`` every window is normalised on its own; d2 is then the squared
    distance between normalised windows and distance = distance_raw = sqrt(d2)."""
    T = _f32(T)
    m = T.size
    if n < 1 or m < 2 * n:
        raise OracleError("need n >= 1 and m >= 2n")
    N = m - n + 1
    idx, nnj = ctypes.c_int64(), ctypes.c_int64()
    d2, mu, sd = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    prof = np.empty(N, dtype=np.float64) if profile else None
    pj = np.empty(N, dtype=np.int64) if profile else None
    fn = load().orc_discord_z if znorm else load().orc_discord
    st = fn(_ptr(T, ctypes.c_float), m, n, _threads(threads),
                            ctypes.byref(idx), ctypes.byref(nnj), ctypes.byref(d2),
                            ctypes.byref(mu), ctypes.byref(sd),
                            _ptr(prof, ctypes.c_double) if profile else None,
                            _ptr(pj, ctypes.c_int64) if profile else None)
    if st == -2:
        raise OracleError("sigma == 0: eq. (2) is undefined for a constant series")
    if st != 0:
        raise OracleError("invalid series")
    dist = math.sqrt(d2.value) if znorm else math.sqrt(d2.value) / sd.value
    out = dict(index=idx.value, nn_index=nnj.value, d2=d2.value,
               distance_raw=math.sqrt(d2.value), distance=dist, mu=mu.value, sigma=sd.value)
    if profile:
        out["profile"] = prof
        out["profile_j"] = pj
    return out


def witness_check(T, n: int, idx: int, d2: float, wit, threads=None, znorm: bool = False):
    """FP64 certificate (see discord_ref.c).  Returns (bad_rows, first_bad,
    exact NN d^2 of idx)."""
    T = _f32(T)
    wit = np.ascontiguousarray(wit, dtype=np.int64)
    N = T.size - n + 1
    if wit.size != N:
        raise OracleError("one witness per row expected")
    fb, nn = ctypes.c_int64(), ctypes.c_double()
    fn = load().orc_witness_check_z if znorm else load().orc_witness_check
    bad = fn(_ptr(T, ctypes.c_float), T.size, n, int(idx), float(d2),
             _ptr(wit, ctypes.c_int64), _threads(threads), ctypes.byref(fb), ctypes.byref(nn))
    if bad < 0:
        raise OracleError("invalid arguments")
    return int(bad), int(fb.value), nn.value


# ----------------------------------------------------------------------------
# SAX preparation (section 3.1)
# ----------------------------------------------------------------------------

def breakpoints(alpha: int = 4) -> np.ndarray:
    """Inner breakpoints beta_1..beta_{alpha-1} of eq. (4): the N(0,1) quantiles
    that cut the real line into alpha equiprobable intervals."""
    nd = statistics.NormalDist(0.0, 1.0)
    return np.array([nd.inv_cdf(k / alpha) for k in range(1, alpha)], dtype=np.float64)


def sax_words(T, n: int, w: int = 4, alpha: int = 4, threads=None,
              znorm: bool = False) -> np.ndarray:
    """Word id of every row: PAA (eq. 3) -> SAX (eq. 4) -> hash (eq. 9), on the
    z-normalised series of eq. (2) (with ``znorm``, on every window normalised
    on its own).  C, sequential sums."""
    T = _f32(T)
    mu, sd = stats(T)
    N = T.size - n + 1
    bp = breakpoints(alpha)
    words = np.empty(N, dtype=np.int32)
    if znorm:
        zmu, zsg = row_zstats(T, n)
        st = load().orc_sax_words_z(_ptr(T, ctypes.c_float), T.size, n, w, alpha,
                                    _ptr(bp, ctypes.c_double), _ptr(zmu, ctypes.c_double),
                                    _ptr(zsg, ctypes.c_double), _ptr(words, ctypes.c_int32),
                                    _threads(threads))
    else:
        st = load().orc_sax_words(_ptr(T, ctypes.c_float), T.size, n, w, alpha,
                                  _ptr(bp, ctypes.c_double), mu, sd,
                                  _ptr(words, ctypes.c_int32), _threads(threads))
    if st != 0:
        raise OracleError("invalid SAX arguments")
    return words


def np_sax_words(T, n: int, w: int = 4, alpha: int = 4) -> np.ndarray:
    """Independent NumPy version of ``sax_words`` (same definitions)."""
    t = np.asarray(T, dtype=np.float32).astype(np.float64)
    mu = t.mean()
    sd = math.sqrt(((t - mu) ** 2).mean())
    z = (t - mu) / sd
    W = np.lib.stride_tricks.sliding_window_view(z, n)
    bp = breakpoints(alpha)
    code = np.zeros(W.shape[0], dtype=np.int64)
    for s in range(w):
        a, b = (s * n) // w, ((s + 1) * n) // w
        paa = W[:, a:b].sum(axis=1) / (b - a)
        sym = np.searchsorted(bp, paa, side="right")   # beta_{k} <= v < beta_{k+1}
        code = code * alpha + sym
    return code.astype(np.int32)


def freq_cand(words, dict_size: int = 256):
    """Eqs. (7)-(8): histogram of word ids, and Cand = ascending rows whose word
    has the minimum frequency among the words that occur."""
    words = np.asarray(words)
    hist = np.bincount(words, minlength=dict_size).astype(np.int64)
    freq = hist[words]
    cand = np.flatnonzero(freq == freq.min()).astype(np.int64)
    return hist, cand


def index_word(words, dict_size: int = 256):
    """Eq. (10) as a CSR inverted index: offsets[dict_size+1] and members[N],
    members of each word in ascending row order."""
    words = np.asarray(words)
    hist = np.bincount(words, minlength=dict_size)
    offsets = np.zeros(dict_size + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(hist)
    members = np.argsort(words, kind="stable").astype(np.int64)
    return offsets, members


# ----------------------------------------------------------------------------
# Independent companions used to pin the C brute force
# ----------------------------------------------------------------------------

def np_discord(T, n: int, block: int = 64) -> dict:
    """NumPy all-pairs brute force (independent of the C code)."""
    t = np.asarray(T, dtype=np.float32).astype(np.float64)
    m = t.size
    if n < 1 or m < 2 * n:
        raise OracleError("need n >= 1 and m >= 2n")
    W = np.lib.stride_tricks.sliding_window_view(t, n)
    N = W.shape[0]
    prof = np.full(N, np.inf)
    pj = np.full(N, -1, dtype=np.int64)
    cols = np.arange(N)
    for r0 in range(0, N, block):
        R = W[r0:r0 + block]
        D = ((R[:, None, :] - W[None, :, :]) ** 2).sum(axis=2)
        rows = np.arange(r0, r0 + R.shape[0])
        D[np.abs(rows[:, None] - cols[None, :]) < n] = np.inf
        pj[r0:r0 + R.shape[0]] = np.argmin(D, axis=1)
        prof[r0:r0 + R.shape[0]] = D[np.arange(R.shape[0]), pj[r0:r0 + R.shape[0]]]
    has = np.isfinite(prof)
    pj[~has] = -1
    best = np.max(prof[has])
    idx = int(np.flatnonzero(has & (prof == best))[0])
    sd = math.sqrt(((t - t.mean()) ** 2).mean())
    return dict(index=idx, nn_index=int(pj[idx]), d2=float(best), profile=prof,
                profile_j=pj, distance=math.sqrt(best) / sd)


def np_discord_z(T, n: int, block: int = 64) -> dict:
    """NumPy all-pairs brute force under per-window normalisation (independent
    of the C code): the normalised window matrix X is built with NumPy's mean
    and std, a flat window becoming zeros, then direct-form distances."""
    t = np.asarray(T, dtype=np.float32).astype(np.float64)
    m = t.size
    if n < 1 or m < 2 * n:
        raise OracleError("need n >= 1 and m >= 2n")
    W = np.lib.stride_tricks.sliding_window_view(t, n)
    mu = W.mean(axis=1, keepdims=True)
    sd = W.std(axis=1, keepdims=True)
    X = np.where(sd > 0, (W - mu) / np.where(sd > 0, sd, 1.0), 0.0)
    N = X.shape[0]
    prof = np.full(N, np.inf)
    pj = np.full(N, -1, dtype=np.int64)
    cols = np.arange(N)
    for r0 in range(0, N, block):
        R = X[r0:r0 + block]
        D = ((R[:, None, :] - X[None, :, :]) ** 2).sum(axis=2)
        rows = np.arange(r0, r0 + R.shape[0])
        D[np.abs(rows[:, None] - cols[None, :]) < n] = np.inf
        pj[r0:r0 + R.shape[0]] = np.argmin(D, axis=1)
        prof[r0:r0 + R.shape[0]] = D[np.arange(R.shape[0]), pj[r0:r0 + R.shape[0]]]
    has = np.isfinite(prof)
    pj[~has] = -1
    best = np.max(prof[has])
    idx = int(np.flatnonzero(has & (prof == best))[0])
    return dict(index=idx, nn_index=int(pj[idx]), d2=float(best), profile=prof,
                profile_j=pj, distance=math.sqrt(best))


def exact_z_profile(values, n: int, digits: int = 60):
    """Per-window normalised NN profile from exact rational arithmetic: with
    integer (or rational) values, C_ij = sum (a - mean a)(b - mean b) and
    V_i = sum (a - mean a)^2 are exact Fractions and
        d^2(i, j) = V_i/s_i^2 + V_j/s_j^2 - 2 C_ij/(s_i s_j),  s_i = sqrt(V_i / n),
    i.e. 2n - 2 C_ij sqrt(n^2 / (V_i V_j)) for non-flat windows (n for one flat
    window, 0 for two).  The one square root is taken in ``digits``-digit decimal
    arithmetic.  Returns (profile, profile_j) as lists of Decimal and int."""
    import decimal
    from fractions import Fraction
    vals = [Fraction(v) for v in values]
    m = len(vals)
    N = m - n + 1
    ctx = decimal.Context(prec=digits)
    wins = []
    for i in range(N):
        w = vals[i:i + n]
        mean = sum(w) / n
        c = [x - mean for x in w]
        wins.append((c, sum(x * x for x in c)))

    def dec(fr):
        return ctx.divide(decimal.Decimal(fr.numerator), decimal.Decimal(fr.denominator))

    prof, pj = [None] * N, [-1] * N
    for i in range(N):
        ci, vi = wins[i]
        for j in range(N):
            if abs(i - j) < n:
                continue
            cj, vj = wins[j]
            if vi == 0 and vj == 0:
                d = decimal.Decimal(0)
            elif vi == 0 or vj == 0:
                d = decimal.Decimal(n)
            else:
                cij = sum(a * b for a, b in zip(ci, cj))
                r = ctx.sqrt(dec(Fraction(n * n) / (vi * vj)))
                d = ctx.subtract(decimal.Decimal(2 * n), ctx.multiply(2 * dec(cij), r))
            if prof[i] is None or d < prof[i]:
                prof[i], pj[i] = d, j
    return prof, pj


def int_discord(values, n: int):
    """Exact enumerator over Python integers: every squared distance is an exact
    integer, so ties are exact.  Returns (index, nn_index, d2, profile)."""
    vals = [int(v) for v in values]
    m = len(vals)
    if n < 1 or m < 2 * n:
        raise OracleError("need n >= 1 and m >= 2n")
    N = m - n + 1
    prof = [None] * N
    pj = [-1] * N
    for i in range(N):
        for j in range(N):
            if abs(i - j) < n:
                continue
            d = 0
            for k in range(n):
                e = vals[i + k] - vals[j + k]
                d += e * e
            if prof[i] is None or d < prof[i]:
                prof[i], pj[i] = d, j
    best_i = None
    for i in range(N):
        if prof[i] is None:
            continue
        if best_i is None or prof[i] > prof[best_i]:
            best_i = i
    return best_i, pj[best_i], prof[best_i], prof


def _pair_table(T, n: int) -> np.ndarray:
    """Squared distance of eq. (1) for every pair of windows, FP64.  np.cumsum
    adds strictly left to right, so its last entry is the sequential sum over
    k = 0..n-1, the value the C brute force computes (small inputs only:
    N x N x n doubles)."""
    t = np.asarray(T, dtype=np.float32).astype(np.float64)
    W = np.lib.stride_tricks.sliding_window_view(t, n)
    diff = W[:, None, :] - W[None, :, :]
    return np.cumsum(diff * diff, axis=2)[:, :, -1]


def _pruned_search(D, n: int, outer, inner):
    """Exact discord search with early abandon, over a table of all squared
    distances (section 2.2).  A row's non-self columns are taken in the order
    ``inner(i)``; the row is abandoned at the first distance strictly below
    the best-so-far (it cannot be the discord, since its NN is smaller still),
    so the distances evaluated for it are those up to and including that one.
    A row that is not abandoned has its NN as the minimum over all of them and
    replaces the best-so-far when larger (lowest index on equal values).  The
    best-so-far starts at 0 with no position.  Returns (index, d2, evaluated)."""
    N = D.shape[0]
    bsf, pos, evals = 0.0, -1, 0
    for i in outer:
        i = int(i)
        cols = np.array([int(j) for j in inner(i) if abs(i - int(j)) >= n], dtype=np.int64)
        if cols.size == 0:
            continue                                   # no non-self match: no NN
        d = D[i, cols]
        below = np.flatnonzero(d < bsf)
        if below.size:
            evals += int(below[0]) + 1
            continue
        evals += cols.size
        nn = float(d.min())
        if pos < 0 or nn > bsf or (nn == bsf and i < pos):
            bsf, pos = nn, i
    return pos, bsf, evals


def alg1(T, n: int, outer=None, inner=None, count: list | None = None):
    """HOTSAX discord search (Algorithm 1, section 2.2) for any visiting order:
    rows in the ``outer`` order, each row's columns in the ``inner(i)`` order
    (matrix order by default), early abandon against the best-so-far, squared
    distances on raw values.  Returns (index, d2); ``count`` (a one-element
    list) receives the number of distances evaluated."""
    D = _pair_table(T, n)
    N = D.shape[0]
    outer = range(N) if outer is None else outer
    pos, bsf, evals = _pruned_search(D, n, outer, inner if inner else (lambda i: range(N)))
    if count is not None:
        count.append(evals)
    return pos, bsf


def phidd(T, n: int, w: int = 4, alpha: int = 4, count: list | None = None):
    """PhiDD (Algorithms 2-4, section 3.2), sequential, on raw values.  The
    preparation gives SAX words, Cand (eq. 7) and Index_Word (eq. 10); the
    method is then the abandoning search above with PhiDD's visiting orders:
    rows of Cand first (PotentialDiscord), then every other row
    (RefineDiscord); each row's columns start with the members of its own word
    (Index_Word) and continue with every other column in matrix order.
    Returns (index, d2)."""
    D = _pair_table(T, n)
    N = D.shape[0]
    words = sax_words(T, n, w, alpha)
    hist, cand = freq_cand(words, alpha ** w)
    offsets, members = index_word(words, alpha ** w)
    in_cand = np.zeros(N, dtype=bool)
    in_cand[cand] = True
    outer = np.concatenate([cand, np.flatnonzero(~in_cand)])

    def inner(i):
        wd = words[i]
        same = members[offsets[wd]:offsets[wd + 1]]
        return np.concatenate([same, np.flatnonzero(words != wd)])

    pos, bsf, evals = _pruned_search(D, n, outer, inner)
    if count is not None:
        count.append(evals)
    return pos, bsf
