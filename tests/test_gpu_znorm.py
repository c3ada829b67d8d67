"""GPU parity of the per-window normalisation mode (opts.znorm = 1).

Algorithm 2 applies Znormalize to the subsequence matrix; read row by row,
every window is normalised by its own mean and standard deviation (eq. (2)
over the window) before the distance of eq. (1) is taken, and a flat window
becomes the zero vector.  The oracle's ``znorm=True`` mode is that definition
written out in FP64 (pinned in test_oracle_znorm_pins.py).  Bars as for the
global mode: discord and neighbour indices bit-exact, the FP64 squared
distance within 1e-9 relative (the certification divides and sums in the
oracle's order, so it is normally bit-identical), preparation arrays exact.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1901_00155_amd import workloads

pytestmark = pytest.mark.gpu

REL = 1e-9
PRECS = ["fp32", "bf16x3"]


def _assert_same(r, ref, ctx=""):
    assert r.index == ref["index"], (ctx, r.index, ref["index"])
    assert r.nn_index == ref["nn_index"], (ctx, r.nn_index, ref["nn_index"])
    assert abs(r.d2 - ref["d2"]) <= REL * ref["d2"], (ctx, r.d2, ref["d2"])
    assert abs(r.distance - ref["distance"]) <= REL * max(ref["distance"], 1e-300), ctx
    assert r.distance == r.distance_raw
    assert r.certified == 1


def _flat_runs(m, seed):
    """Random walk with flat stretches (windows inside them have sigma = 0) and
    exact repeats (distance-0 neighbours)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.standard_normal(m))
    for _ in range(4):
        a = int(rng.integers(0, m - 40))
        t[a:a + int(rng.integers(10, 40))] = t[a]
    b = int(rng.integers(0, m // 2 - 30))
    t[m // 2:m // 2 + 30] = t[b:b + 30]
    return t.astype(np.float32)


@pytest.mark.parametrize("case", ["small", "rw3000_n37", "flat900_n12"])
def test_znorm_preparation_matches_oracle(gpu, case):
    if case == "small":
        w = workloads.small()
        T, n = w.series, w.n
    elif case == "rw3000_n37":
        T, n = workloads.random_walk(3000, seed=3000), 37
    else:
        T, n = _flat_runs(900, 5), 12
    zmu, zsg = oracle.row_zstats(T, n)
    with gpu.Plan(T, n, znorm=True) as p:
        assert np.array_equal(p.copy("row_mean"), zmu)
        assert np.array_equal(p.copy("row_sigma"), zsg)
        words = oracle.sax_words(T, n, znorm=True)
        assert np.array_equal(p.copy("words"), words)
        hist, cand = oracle.freq_cand(words)
        assert np.array_equal(p.copy("hist"), hist[:256])
        assert np.array_equal(p.copy("cand"), cand)
        off, mem = oracle.index_word(words)
        assert np.array_equal(p.copy("csr_offsets"), off)
        assert np.array_equal(p.copy("csr_members"), mem)
    if case == "flat900_n12":
        assert np.any(zsg == 0.0)


def test_row_sigma_needs_znorm(gpu):
    with gpu.Plan(workloads.random_walk(500, seed=1), 10) as p:
        with pytest.raises(gpu.DiscordError):
            p.copy("row_sigma")


ZCASES = [
    (16, 1, 0), (40, 3, 1), (64, 32, 2), (100, 7, 4), (257, 9, 5), (300, 64, 6),
    (513, 100, 7), (1001, 333, 9), (2049, 17, 10), (3000, 128, 11),
    (4100, 200, 12), (4096, 64, 14), (1500, 512, 15), (2600, 280, 16),
    # windows beyond 512 (the split-BF16 scan with operands built from the series)
    (2600, 528, 23), (3600, 700, 26), (4500, 2048, 20),
]


@pytest.mark.parametrize("m,n,seed", ZCASES)
@pytest.mark.parametrize("mode", ["full", "abandon-matrix", "abandon-phidd", "abandon-near"])
@pytest.mark.parametrize("precision", PRECS)
def test_znorm_discord_matches_oracle(gpu, m, n, seed, mode, precision):
    T = workloads.random_walk(m, seed=seed)
    ref = oracle.discord(T, n, znorm=True)
    order = {"full": 1, "abandon-matrix": 0, "abandon-phidd": 1, "abandon-near": 2}[mode]
    with gpu.Plan(T, n, abandon=mode != "full", order=order, precision=precision,
                  znorm=True) as p:
        r = p.search()
    _assert_same(r, ref, (m, n, seed, mode))


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("precision", PRECS)
def test_znorm_flat_windows_and_repeats(gpu, seed, precision):
    """Flat windows (zero vectors after normalisation, distance n to any other
    non-flat window and 0 to each other) and exact repeats (distance 0)."""
    m = 700 + 150 * seed
    n = [8, 12, 20, 33][seed]
    T = _flat_runs(m, 40 + seed)
    ref = oracle.discord(T, n, znorm=True)
    with gpu.Plan(T, n, precision=precision, znorm=True) as p:
        r = p.search()
        wit = p.copy("nn_witness")
    _assert_same(r, ref, (m, n))
    bad, first, _ = oracle.witness_check(T, n, r.index, r.d2, wit, znorm=True)
    assert bad == 0, first


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("precision", PRECS)
def test_znorm_integer_series(gpu, seed, precision):
    """Small-alphabet integer series: many exactly repeated and flat windows,
    so exact ties are common and the lowest-index rules decide."""
    rng = np.random.default_rng(700 + seed)
    m = int(rng.integers(60, 500))
    n = int(rng.integers(2, 10))
    T = rng.integers(-2, 3, m).astype(np.float32)
    ref = oracle.discord(T, n, znorm=True)
    with gpu.Plan(T, n, precision=precision, znorm=True) as p:
        _assert_same(p.search(), ref, (m, n))


def test_znorm_rows_nn_fp64_bit_exact(gpu):
    T = _flat_runs(5000, 77)
    n = 50
    rows = np.array([0, 1, 49, 50, 2500, 2510, 4000, 4901, 4950], dtype=np.int64)
    d_ref, j_ref = oracle.rows_nn(T, n, rows, znorm=True)
    with gpu.Plan(T, n, znorm=True) as p:
        d, j = p.rows_nn_fp64(rows)
    assert np.array_equal(j, j_ref)
    assert np.array_equal(d, d_ref)


@pytest.mark.parametrize("precision", PRECS)
def test_znorm_small_workload_and_scale_invariance(gpu, precision):
    """The small workload, and the same series under an affine map a T + b: the
    per-window normalisation removes it exactly in real arithmetic, so the
    discord row is unchanged and the distance agrees to rounding."""
    w = workloads.small()
    ref = oracle.discord(w.series, w.n, znorm=True)
    with gpu.Plan(w.series, w.n, precision=precision, znorm=True) as p:
        r = p.search()
    _assert_same(r, ref)
    T2 = (w.series.astype(np.float64) * 4.0 + 1000.0).astype(np.float32)
    ref2 = oracle.discord(T2, w.n, znorm=True)
    with gpu.Plan(T2, w.n, precision=precision, znorm=True) as p:
        r2 = p.search()
    _assert_same(r2, ref2)
    assert r2.index == r.index
    assert math.isclose(r2.distance, r.distance, rel_tol=1e-4)


def test_znorm_fp32_full_scan_profile(gpu):
    """FP32 normalised-form minima: within the absolute rounding bound of the
    form q_i + q_j - 2 C s_i s_j of the exact NN; witnesses are non-self."""
    m, n = 3000, 64
    T = workloads.random_walk(m, seed=31)
    ref = oracle.discord(T, n, profile=True, znorm=True)
    with gpu.Plan(T, n, abandon=False, znorm=True) as p:
        r = p.search()
        approx = p.copy("nn_approx").astype(np.float64)
        wit = p.copy("nn_witness")
    _assert_same(r, ref)
    bound = (2.2 * (n + 4) * n + 16 * n) * 2.0 ** -24
    assert np.all(np.abs(approx - ref["profile"]) <= bound)
    N = m - n + 1
    assert np.all(np.abs(np.arange(N) - wit) >= n)


@pytest.mark.parametrize("m,n", [(3000, 64), (2600, 528), (3333, 1500), (4500, 2048)])
def test_znorm_bf16x3_full_scan_profile(gpu, m, n):
    """Split-BF16 normalised minima: within 2^-12 * 2n of the exact NN
    (normalised windows have squared norm n, and the split products carry
    ~2^-16 of |a'||b'|); witnesses are non-self and the result is certified."""
    T = workloads.random_walk(m, seed=m + n)
    ref = oracle.discord(T, n, profile=True, znorm=True)
    with gpu.Plan(T, n, precision="bf16x3", abandon=False, znorm=True) as p:
        r = p.search()
        approx = p.copy("nn_approx").astype(np.float64)
        wit = p.copy("nn_witness")
    _assert_same(r, ref)
    prof = ref["profile"]
    fin = np.isfinite(prof)   # rows with no non-self match: infinite on both sides
    assert np.array_equal(np.isfinite(approx), fin)
    assert np.all(np.abs(approx[fin] - prof[fin]) <= 2.0 ** -12 * 2 * n)
    N = m - n + 1
    assert np.all(np.abs(np.arange(N) - wit)[fin] >= n)


def _certify_z(w, r, wit):
    bad, first, nn = oracle.witness_check(w.series, w.n, r.index, r.d2, wit, znorm=True)
    assert bad == 0, first
    assert abs(r.d2 - nn) <= REL * nn


def test_znorm_walk1m_certificate_both_precisions(gpu):
    """m = 2^20, n = 128 with four planted anomalies, per-window normalisation:
    both precisions give the same discord, certified in FP64 against every
    row's witness by the oracle."""
    w = workloads.walk1m()
    out = {}
    for precision in PRECS:
        with gpu.Plan(w.series, w.n, precision=precision, znorm=True) as p:
            r = p.search()
            wit = p.copy("nn_witness")
        _certify_z(w, r, wit)
        out[precision] = (r.index, r.nn_index, r.d2)
        print(precision, r.index, r.d2, r.pairs_evaluated, r.ms_search, r.rows_rescored,
              [a[0] for a in w.anomalies], flush=True)
    assert out["fp32"] == out["bf16x3"], out
