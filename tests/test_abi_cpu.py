"""The C-ABI library loads on the CPU host and exports every symbol the public
header declares.  No compute call is made here (no GPU in this container);
only host-side helpers run."""
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "discord.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(discord_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def dd():
    import paper_1901_00155_amd as dd
    if not os.path.exists(dd.LIB_PATH):
        pytest.fail("libdiscord.so is not built: run __graft_entry__.build()")
    dd.load()
    return dd


def test_every_declared_symbol_is_exported(dd):
    lib = dd.load()
    names = _declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(dd.EXPORTED) == names


def test_opts_defaults_and_workspace(dd):
    o = dd.default_opts()
    assert (o.precision, o.abandon, o.order, o.paa_w, o.alphabet) == (0, 1, 2, 4, 4)
    assert dd.load().discord_abi_version() == dd.ABI_VERSION == 4
    assert dd.workspace_bytes(4096, 64) > 4 * 4096
    assert dd.workspace_bytes(100, 64) == 0            # m < 2n
    assert dd.workspace_bytes(4096, 64, paa_w=9) == 0  # bad option
    assert o.znorm == 0                                 # eq. (2) over the whole series


def test_znorm_option_workspace(dd):
    """Per-window normalisation adds the FP64 row standard deviations and the
    FP32 row scales (N + 64 entries) to the plan and drops the mean-gap bound
    arrays of global normalisation (4 B per row, 2 x (65536 bins + 4096 groups
    + 256 supergroups), the range); other values are refused."""
    m, n = 4096, 64
    N = m - n + 1
    base = dd.workspace_bytes(m, n)
    z = dd.workspace_bytes(m, n, znorm=1)
    bound = 4 * N + 16 + 2 * 4 * (65536 + 4096 + 256)
    assert z >= base - bound - 4 * 256 + 8 * N + 4 * (N + 64)
    assert z <= base - bound + 8 * N + 4 * (N + 64) + 4 * 256
    assert dd.workspace_bytes(m, n, znorm=2) == 0
    assert dd.workspace_bytes(m, n, znorm=-1) == 0


def test_sax_breakpoints_match_oracle(dd):
    """The library's eq. (4) breakpoints (Newton on erfc) against the oracle's
    (statistics.NormalDist): identical for |A| = 4, within one ulp otherwise."""
    assert np.array_equal(dd.sax_breakpoints(4), oracle.breakpoints(4))
    for a in range(2, 9):
        np.testing.assert_allclose(dd.sax_breakpoints(a), oracle.breakpoints(a), rtol=0, atol=4e-16)


def test_strerror(dd):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert dd.strerror(code)


def test_visiting_order_option(dd):
    assert dd.workspace_bytes(4096, 64, order=2) > 0
    assert dd.workspace_bytes(4096, 64, order=3) == 0


def test_near_first_order_covers_every_needed_block(tmp_path):
    """tests/native/spiral_check.cpp: exhaustive check of the near-first column
    order of the scan kernels (csrc/spiral.hpp) on small sizes."""
    import shutil
    import subprocess
    cxx = shutil.which("g++") or shutil.which("c++")
    if not cxx:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "spiral_check")
    subprocess.run([cxx, "-std=c++17", "-O2", os.path.join(ROOT, "tests", "native", "spiral_check.cpp"),
                    "-o", exe], check=True, timeout=120)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "OK" in r.stdout, r.stdout + r.stderr


def test_library_has_no_unresolved_internal_symbols(dd):
    """Every internal function the library calls is linked in (a source file
    missing from the build would leave an undefined dd:: symbol)."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if not nm:
        pytest.skip("nm not available")
    out = subprocess.run([nm, "-uC", dd.LIB_PATH], capture_output=True, text=True, check=True).stdout
    assert "dd::" not in out, [ln for ln in out.splitlines() if "dd::" in ln]


def test_binding_constants_match_header():
    import re
    from paper_1901_00155_amd import _binding as B
    text = open(HEADER).read()
    assert int(re.search(r"#define DISCORD_MIXED_MAX_N (\d+)", text).group(1)) == B.MIXED_MAX_N


@pytest.mark.parametrize("total,xccs", [(256, 8), (304, 8), (64, 2), (40, 1), (32, 4)])
def test_cu_mask_is_balanced_over_dies(dd, total, xccs):
    """Every die keeps cus / xccs CUs under both the contiguous (bit b on die
    b // per) and the interleaved (bit b on die b % xccs) assignment, no bit
    lies beyond the device's CUs, and no bit repeats."""
    per = total // xccs
    for cus in range(xccs, total + 1, xccs):
        if per % xccs:
            with pytest.raises(dd.DiscordError):
                dd.cu_mask(total, xccs, cus)
            return
        words = dd.cu_mask(total, xccs, cus)
        assert len(words) == (total + 31) // 32
        bits = [b for b in range(32 * len(words)) if (words[b // 32] >> (b % 32)) & 1]
        assert len(bits) == cus and max(bits) < total
        for die in range(xccs):
            assert sum(1 for b in bits if b // per == die) == cus // xccs
            assert sum(1 for b in bits if b % xccs == die) == cus // xccs


def test_cu_mask_rejects_bad_sizes(dd):
    for args in [(256, 8, 0), (256, 8, 12), (256, 8, 264), (256, 0, 8), (250, 8, 8), (0, 1, 1)]:
        with pytest.raises(dd.DiscordError):
            dd.cu_mask(*args)


@pytest.mark.parametrize("m,n", [(4096, 64), (50000, 512), (50000, 600), (100000, 2048)])
def test_split_bf16_workspace_is_linear_in_the_series(dd, m, n):
    """A split-BF16 plan builds its operands from the series as it scans, so it
    holds no per-window matrix: its footprint is the FP32 plan's plus O(N)
    FP32 row statistics, whatever the window.  Windows up to
    DISCORD_MIXED_MAX_N are accepted and longer ones refused."""
    N = m - n + 1
    f32 = dd.workspace_bytes(m, n)
    b16 = dd.workspace_bytes(m, n, precision="bf16x3")
    assert f32 > 0 and b16 >= f32
    assert b16 - f32 < 16 * N + (1 << 20)
    assert dd.workspace_bytes(2 * (dd.MIXED_MAX_N + 1), dd.MIXED_MAX_N + 1,
                              precision="bf16x3") == 0


def test_noalloc_refuses_plans_beyond_its_static_workspace(dd):
    """The allocation-free entry point checks the plan's size against its
    static workspace before any device call, so the refusal is visible here
    without a GPU; the limit matches the header."""
    import re
    hdr = open(os.path.join(os.path.dirname(dd.LIB_PATH), "..", "..", "include",
                            "discord.h")).read()
    assert re.search(r"DISCORD_NOALLOC_MAX_BYTES \(\(size_t\)32 << 20\)", hdr)
    assert dd.NOALLOC_MAX_BYTES == 32 << 20
    m, n = 1 << 20, 128
    assert dd.workspace_bytes(m, n) > dd.NOALLOC_MAX_BYTES
    T = np.zeros(m, dtype=np.float32)
    with pytest.raises(dd.DiscordError) as e:
        dd.search_series_noalloc(T, n)
    assert e.value.status == -6 and "static workspace" in str(e.value)
    # a split-BF16 plan holds no per-window matrix: a 2^16-point plan fits the
    # static workspace in both precisions, the 2^20-point one in neither
    m2 = 1 << 16
    assert dd.workspace_bytes(m2, 256) <= dd.NOALLOC_MAX_BYTES
    assert dd.workspace_bytes(m2, 256, precision="bf16x3") <= dd.NOALLOC_MAX_BYTES
    assert dd.workspace_bytes(m, n, precision="bf16x3") > dd.NOALLOC_MAX_BYTES
    with pytest.raises(dd.DiscordError) as e:
        dd.search_series_noalloc(T, n, precision="bf16x3")
    assert e.value.status == -6


def test_search_once_refuses_bad_arguments_before_any_device_call(dd):
    """discord_search_once checks its arguments and the caller's workspace
    (size against discord_workspace_bytes, 256-byte alignment) before it makes
    any device call, so each refusal is visible here without a GPU."""
    import ctypes
    lib = dd.load()
    m, n = 4096, 64
    T = np.zeros(m, dtype=np.float32)
    tp = ctypes.c_void_p(T.ctypes.data)
    opts = dd.default_opts()
    need = lib.discord_workspace_bytes(m, n, ctypes.byref(opts))
    assert need > 0
    r = dd.Result()
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: every call below is refused first
    # no result struct; window too long (2n > m); empty window
    assert lib.discord_search_once(tp, m, n, ctypes.byref(opts), fake, need, None, None) == -1
    assert lib.discord_search_once(tp, m, m // 2 + 1, ctypes.byref(opts), fake, need, None,
                                   ctypes.byref(r)) == -1
    assert lib.discord_search_once(tp, m, 0, ctypes.byref(opts), fake, need, None,
                                   ctypes.byref(r)) == -1
    # split-BF16 beyond its longest window
    big = dd.MIXED_MAX_N + 1
    ob = dd.default_opts(precision="bf16x3")
    Tb = np.zeros(2 * big, dtype=np.float32)
    assert lib.discord_search_once(ctypes.c_void_p(Tb.ctypes.data), Tb.size, big,
                                   ctypes.byref(ob), fake, need, None, ctypes.byref(r)) == -6
    # a workspace one granule short, and a misaligned one
    for ptr, size in ((1 << 20, need - 256), ((1 << 20) + 4, need)):
        st = lib.discord_search_once(tp, m, n, ctypes.byref(opts), ctypes.c_void_p(ptr), size,
                                     None, ctypes.byref(r))
        assert st == -3, st
        msg = lib.discord_plan_error(None).decode()
        assert "needs" in msg and str(need) in msg
