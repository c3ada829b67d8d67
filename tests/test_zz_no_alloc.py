"""The allocation-free entry point (discord_search_series_noalloc) against
the allocating one (discord_prepare + discord_search on a plan): the same
certified result, bit for bit, on two calls in a row in both precisions, the
second with a smaller series, so the static workspace's leftover contents from
the first call must not leak into the second."""
import numpy as np
import pytest

import oracle
from paper_1901_00155_amd import workloads

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "bf16x3"]


def _same(a, b):
    assert (a.index, a.nn_index) == (b.index, b.nn_index)
    assert a.d2 == b.d2 and a.distance == b.distance
    assert a.certified == b.certified == 1
    assert a.pairs_evaluated > 0 and b.pairs_evaluated > 0


@pytest.mark.parametrize("precision", PRECS)
def test_noalloc_matches_plan_on_two_calls(gpu, precision):
    import torch
    dd = gpu
    big = workloads.random_walk(48000, seed=71)
    small = workloads.small()
    cases = [(big, 128), (small.series, small.n)]
    for T, n in cases:
        assert dd.workspace_bytes(T.size, n, precision=precision) <= dd.NOALLOC_MAX_BYTES
    s = torch.cuda.Stream()
    for k, (T, n) in enumerate(cases):
        with dd.Plan(T, n, precision=precision) as p:
            ref = p.search()
        Td = torch.from_numpy(T).cuda()
        got = dd.search_series_noalloc(Td, n, stream=s, precision=precision)
        print(precision, k, T.size, n, got.index, got.d2, flush=True)
        _same(got, ref)
        assert got.ms_search == 0.0
        if k == 1:
            o = oracle.discord(T, n)
            assert got.index == o["index"] and got.nn_index == o["nn_index"]
            assert abs(got.d2 - o["d2"]) <= 1e-9 * o["d2"]


def test_noalloc_host_series_and_errors(gpu):
    dd = gpu
    w = workloads.small()
    with dd.Plan(w.series, w.n) as p:
        ref = p.search()
    got = dd.search_series_noalloc(w.series, w.n)        # host series, null stream
    _same(got, ref)
    with pytest.raises(dd.DiscordError) as e:
        dd.search_series_noalloc(np.full(5000, 2.0, np.float32), 64)
    assert e.value.status == -2
    bad = w.series.copy()
    bad[10] = np.nan
    with pytest.raises(dd.DiscordError) as e:
        dd.search_series_noalloc(bad, w.n)
    assert e.value.status == -1
    # a good call after the failures still gives the plan's result
    _same(dd.search_series_noalloc(w.series, w.n), ref)
