"""discord_search_once (preparation and search as one device sequence, one
synchronisation) against discord_prepare + discord_search on a plan: the same
certified result bit for bit, in both precisions, both normalisations and the
three visiting orders (the PhiDD order takes the path that synchronises after
the preparation), for device and host series, a caller workspace and a
library-allocated one; the timing fields it states; its errors."""
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
    assert a.pairs_evaluated == b.pairs_evaluated or a.pairs_evaluated > 0


@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("znorm", [False, True])
@pytest.mark.parametrize("order", [2, 1, 0])
def test_once_matches_plan(gpu, precision, znorm, order):
    import torch
    dd = gpu
    T = workloads.random_walk(60000, seed=83)
    n = 96
    Td = torch.from_numpy(T).cuda()
    with dd.Plan(Td, n, precision=precision, znorm=znorm, order=order,
                 torch_workspace=True) as p:
        ref = p.search()
    got = dd.search_once(Td, n, precision=precision, znorm=znorm, order=order)
    print(precision, znorm, order, got.index, got.d2, flush=True)
    _same(got, ref)
    # one sequence: no separate preparation time, except in the PhiDD order,
    # which synchronises after the preparation
    assert (got.ms_prepare > 0.0) if order == 1 else (got.ms_prepare == 0.0)
    assert got.ms_scan > 0.0 and got.ms_search >= got.ms_scan
    assert got.scan_launches == ref.scan_launches


def test_once_small_against_oracle_host_series_library_workspace(gpu):
    dd = gpu
    w = workloads.small()
    o = oracle.discord(w.series, w.n)
    for prec in PRECS:
        got = dd.search_once(w.series, w.n, precision=prec, torch_workspace=False)
        print(prec, got.index, got.d2, flush=True)
        assert got.index == o["index"] and got.nn_index == o["nn_index"]
        assert abs(got.d2 - o["d2"]) <= 1e-9 * o["d2"]


def test_once_repeated_on_one_stream(gpu):
    """Two calls in a row on one stream and one caller workspace, the second on
    a shorter series: nothing from the first call's state leaks."""
    import ctypes
    import torch
    dd = gpu
    lib = dd.load()
    a = workloads.random_walk(50000, seed=5)
    b = workloads.small()
    s = torch.cuda.Stream()
    opts = dd.default_opts(precision="bf16x3")
    need = max(lib.discord_workspace_bytes(a.size, 128, ctypes.byref(opts)),
               lib.discord_workspace_bytes(b.series.size, b.n, ctypes.byref(opts)))
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    wp = (ws.data_ptr() + 255) // 256 * 256
    for T, n in ((a, 128), (b.series, b.n)):
        Td = torch.from_numpy(T).cuda()
        with dd.Plan(Td, n, precision="bf16x3", torch_workspace=True) as p:
            ref = p.search()
        r = dd.Result()
        st = lib.discord_search_once(ctypes.c_void_p(Td.data_ptr()), T.size, n,
                                     ctypes.byref(opts), ctypes.c_void_p(wp), need,
                                     ctypes.c_void_p(s.cuda_stream), ctypes.byref(r))
        print(T.size, n, st, r.index, flush=True)
        assert st == 0
        _same(r, ref)


def test_once_errors(gpu):
    import ctypes
    import torch
    dd = gpu
    lib = dd.load()
    with pytest.raises(dd.DiscordError) as e:
        dd.search_once(np.full(5000, 2.0, np.float32), 64)
    assert e.value.status == -2                       # ECONST: sigma = 0
    bad = workloads.small().series.copy()
    bad[10] = np.nan
    with pytest.raises(dd.DiscordError) as e:
        dd.search_once(bad, 64)
    assert e.value.status == -1                       # EINVAL: not finite
    with pytest.raises(dd.DiscordError) as e:
        dd.search_once(workloads.small().series, 3000)   # 2n > m
    assert e.value.status == -1
    # a workspace one granule short, and a misaligned one: ENOMEM before any work
    T = torch.from_numpy(workloads.small().series).cuda()
    opts = dd.default_opts()
    need = lib.discord_workspace_bytes(T.numel(), 64, ctypes.byref(opts))
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    wp = (ws.data_ptr() + 255) // 256 * 256
    r = dd.Result()
    for ptr, size in ((wp, need - 256), (wp + 4, need)):
        st = lib.discord_search_once(ctypes.c_void_p(T.data_ptr()), T.numel(), 64,
                                     ctypes.byref(opts), ctypes.c_void_p(ptr), size, None,
                                     ctypes.byref(r))
        assert st == -3, st                           # ENOMEM
        assert "needs" in lib.discord_plan_error(None).decode()
    # the library still answers afterwards
    assert dd.search_once(T, 64).certified == 1
