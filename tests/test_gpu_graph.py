"""The search replayed from a HIP graph (discord_search_graph) against the
eager search (discord_search) on the same plan: every replay gives the same
certified result, bit for bit, with eager searches and host synchronisations
between the replays; and the oracle's answer where it is quick."""
import numpy as np
import pytest

import oracle
from paper_1901_00155_amd import workloads

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "bf16x3"]


def _key(r):
    return (r.index, r.nn_index, r.d2, r.distance, r.certified, r.rows_rescored)


@pytest.mark.parametrize("order", [0, 1, 2])
@pytest.mark.parametrize("precision", PRECS)
def test_graph_replays_match_eager(gpu, precision, order):
    import torch
    dd = gpu
    T = workloads.random_walk(20000, seed=55 + order, noise=0.01)
    n = 96
    ref = oracle.discord(T, n)
    with dd.Plan(T, n, precision=precision, order=order) as p:
        eager = p.search()
        assert eager.index == ref["index"] and eager.nn_index == ref["nn_index"]
        for k in range(4):
            g = p.search_graph()
            print(precision, order, k, g.index, g.d2, g.ms_search, flush=True)
            assert _key(g) == _key(eager), k
            torch.cuda.synchronize()
            e = p.search()                        # eager work between the replays
            assert _key(e) == _key(eager), k


@pytest.mark.parametrize("precision", PRECS)
def test_graph_full_scan_and_znorm(gpu, precision):
    dd = gpu
    T = workloads.random_walk(6000, seed=9)
    for kw in ({"abandon": False}, {"znorm": True}):
        with dd.Plan(T, 50, precision=precision, **kw) as p:
            eager = p.search()
            for k in range(3):
                assert _key(p.search_graph()) == _key(eager), (kw, k)


def test_graph_walk1m_certificate(gpu):
    """The default workload (m = 2^20, n = 128) replayed from a graph: the same
    answer as the eager search, and its witness array certifies it."""
    w = workloads.walk1m()
    with gpu.Plan(w.series, w.n) as p:
        eager = p.search()
        for k in range(3):
            g = p.search_graph()
            assert _key(g) == _key(eager)
        wit = p.copy("nn_witness")
    bad, first, nn = oracle.witness_check(w.series, w.n, g.index, g.d2, wit)
    assert bad == 0, first
    assert abs(nn - g.d2) <= 1e-9 * nn
