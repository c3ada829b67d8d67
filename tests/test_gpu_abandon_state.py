"""The approximate state an early-abandon search leaves behind, row by row,
against exact FP64 arithmetic (not only the certified answer, which the FP64
certification would make right whatever the scan did):

- a row the search completed holds its exact NN within the scan's error bound;
- a row that left early holds the distance to its witness within that bound,
  and the witness is a non-self match.

Series and windows are chosen so that the split-BF16 scan runs steps with
one, two, three and four live row blocks in a workgroup (the one-live-block
steps share the columns among the four wavefronts)."""
import numpy as np
import pytest
from numpy.lib.stride_tricks import sliding_window_view

import oracle
from paper_1901_00155_amd import workloads

pytestmark = pytest.mark.gpu

FULL, ABANDONED = 1, 2


def _windows(T, n, znorm):
    W = sliding_window_view(T.astype(np.float64), n)
    if not znorm:
        return W
    mu = W.mean(axis=1, keepdims=True)
    sd = np.sqrt(((W - mu) ** 2).mean(axis=1, keepdims=True))
    Z = np.where(sd > 0, (W - mu) / np.where(sd > 0, sd, 1.0), 0.0)
    return Z


def _state(gpu, T, n, precision, znorm):
    with gpu.Plan(T, n, precision=precision, znorm=znorm) as p:
        r = p.search()
        approx = p.copy("nn_approx").astype(np.float64)
        wit = p.copy("nn_witness").astype(np.int64)
        st = p.copy("row_state")
        cn = p.copy("row_cnorm")
        mean = p.copy("row_mean")
    return r, approx, wit, st, cn, mean


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("znorm", [False, True])
@pytest.mark.parametrize("m,n,seed", [(20000, 96, 3), (16000, 128, 11), (12000, 300, 7)])
def test_abandon_state_rows(gpu, precision, znorm, m, n, seed):
    T = workloads.random_walk(m, seed=seed)
    N = m - n + 1
    ref = oracle.discord(T, n, profile=True, znorm=znorm)
    prof = ref["profile"]
    r, approx, wit, st, cn, mean = _state(gpu, T, n, precision, znorm)
    print(precision, znorm, m, n, r.index, r.pairs_evaluated, np.bincount(st, minlength=3),
          flush=True)
    assert r.index == ref["index"] and r.certified == 1
    assert set(np.unique(st)) <= {FULL, ABANDONED}
    # error bounds per row: FP32 direct form, relative; split-BF16 absolute in
    # the centred norms (block offsets as in the full-scan profile tests), or
    # 2^-12 * 2n for normalised windows
    if precision == "fp32" and znorm:
        # absolute: the form q_i + q_j - 2 C s_i s_j
        ab = (2.2 * (n + 4) * n + 16 * n) * 2.0 ** -24
        tol = lambda exact, rows: np.full(rows.size, ab)   # noqa: E731
    elif precision == "fp32":
        rel = (n + 3) * 2.0 ** -24 * 1.01
        tol = lambda exact, rows: rel * exact + 1e-30   # noqa: E731
    elif znorm:
        tol = lambda exact, rows: np.full(rows.size, 2.0 ** -12 * 2 * n)   # noqa: E731
    else:
        off = mean[np.minimum(np.arange(N) // 128 * 128 + 64, N - 1)].astype(np.float32)
        x2 = cn + n * (mean - off.astype(np.float64)) ** 2
        big = np.max(x2)
        tol = lambda exact, rows: 2.0 ** -12 * (x2[rows] + big) + 1e-6   # noqa: E731
    full = np.flatnonzero((st == FULL) & np.isfinite(prof))
    assert np.all(np.abs(approx[full] - prof[full]) <= tol(prof[full], full))
    left = np.flatnonzero(st == ABANDONED)
    assert left.size > 0
    assert np.all(wit[left] >= 0) and np.all(np.abs(left - wit[left]) >= n)
    Wv = _windows(T, n, znorm)
    exact = ((Wv[left] - Wv[wit[left]]) ** 2).sum(axis=1)
    assert np.all(np.abs(approx[left] - exact) <= tol(exact, left)), (
        np.max(np.abs(approx[left] - exact) - tol(exact, left)))
    # the distance a row left with is never below its exact NN by more than
    # the bound
    assert np.all(approx[left] - prof[left] >= -tol(prof[left], left))
