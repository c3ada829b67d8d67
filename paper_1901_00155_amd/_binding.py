"""ctypes binding of libdiscord.so (include/discord.h).

Argument marshalling only: every step of the search runs in the HIP library.
PyTorch is used for device memory (optional caller workspace, device-resident
series) and streams.  There is no CPU fallback: if the library is missing the
first call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "load", "DiscordError", "Opts", "Result", "Plan", "search", "default_opts",
    "workspace_bytes", "strerror", "sax_breakpoints", "search_series",
    "search_series_noalloc", "search_once", "NOALLOC_MAX_BYTES",
    "FIELD", "PREC_FP32", "PREC_BF16X3", "MIXED_MAX_N", "ABI_VERSION", "LIB_PATH", "EXPORTED", "Server",
    "ServerConfig", "cu_mask", "CULimitedStream",
    "Request", "Completion", "ServerStats", "EXECUTOR_FN",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libdiscord.so")

PREC_FP32 = 0
PREC_BF16X3 = 1
MIXED_MAX_N = 2048  # DISCORD_MIXED_MAX_N: longest window of the split-BF16 scan
ABI_VERSION = 4     # DISCORD_ABI_VERSION of the header these structures mirror
NOALLOC_MAX_BYTES = 32 << 20  # DISCORD_NOALLOC_MAX_BYTES: static workspace per device
_PREC = {"fp32": PREC_FP32, "bf16x3": PREC_BF16X3, PREC_FP32: PREC_FP32, PREC_BF16X3: PREC_BF16X3}

FIELD = {
    "words": (0, np.int32), "hist": (1, np.int32), "cand": (2, np.int32),
    "csr_offsets": (3, np.int32), "csr_members": (4, np.int32),
    "nn_approx": (5, np.float32), "nn_witness": (6, np.int32), "row_state": (7, np.int32),
    "row_mean": (8, np.float64), "row_cnorm": (9, np.float64), "row_sigma": (10, np.float64),
    "row_bound": (11, np.float32),
}

# every symbol the public header declares (checked by the CPU tests)
EXPORTED = [
    "discord_default_opts", "discord_abi_version", "discord_workspace_bytes", "discord_prepare", "discord_search",
    "discord_release", "discord_search_graph", "discord_strerror", "discord_plan_error", "discord_sax_breakpoints",
    "discord_search_series", "discord_search_series_noalloc", "discord_search_once", "discord_plan_count", "discord_plan_copy", "discord_rows_nn_fp64",
    "discord_server_create", "discord_server_create_with_executor", "discord_server_submit",
    "discord_server_poll", "discord_server_get_stats", "discord_server_destroy",
    "discord_cu_mask", "discord_stream_create_cu_limited", "discord_stream_destroy",
]


class DiscordError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("abandon", ctypes.c_int32),
                ("order", ctypes.c_int32), ("paa_w", ctypes.c_int32), ("alphabet", ctypes.c_int32),
                ("probe_steps", ctypes.c_int32), ("znorm", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("index", ctypes.c_int64), ("nn_index", ctypes.c_int64),
                ("d2", ctypes.c_double), ("distance_raw", ctypes.c_double),
                ("distance", ctypes.c_double), ("mu", ctypes.c_double),
                ("sigma", ctypes.c_double), ("max_rel_err", ctypes.c_double),
                ("certified", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("pairs_evaluated", ctypes.c_uint64), ("rows_rescored", ctypes.c_uint64),
                ("rows_abandoned", ctypes.c_uint64), ("cand_rows", ctypes.c_uint64),
                ("ms_prepare", ctypes.c_double), ("ms_search", ctypes.c_double),
                ("ms_scan", ctypes.c_double), ("scan_launches", ctypes.c_uint64),
                ("graph", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("slots", ctypes.c_int32),
                ("max_queued", ctypes.c_int32), ("opts", Opts)]


class Request(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("T", ctypes.POINTER(ctypes.c_float)),
                ("m", ctypes.c_int64), ("n", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("workspace", ctypes.c_void_p), ("ws_offset", ctypes.c_size_t),
                ("ws_bytes", ctypes.c_size_t)]


class Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("ws_offset", ctypes.c_size_t), ("ws_bytes", ctypes.c_size_t),
                ("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double), ("result", Result),
                ("detail", ctypes.c_char * 96)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("result", "detail")}
        d["detail"] = self.detail.decode(errors="replace")
        d["result"] = self.result.as_dict()
        return d


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("queued", ctypes.c_int32), ("running", ctypes.c_int32),
                ("peak_running", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("budget_bytes", ctypes.c_size_t), ("bytes_in_use", ctypes.c_size_t),
                ("peak_bytes_in_use", ctypes.c_size_t), ("busy_ms", ctypes.c_double),
                ("elapsed_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


# int (*)(void* ctx, const discord_request*, const discord_opts*, discord_result*, char*, size_t)
EXECUTOR_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(Request),
                               ctypes.POINTER(Opts), ctypes.POINTER(Result), ctypes.c_void_p,
                               ctypes.c_size_t)

_lib = None


def load():
    """Load libdiscord.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.discord_abi_version.argtypes = []
    lib.discord_abi_version.restype = i32
    got = lib.discord_abi_version()
    if got != ABI_VERSION:
        raise RuntimeError(f"{LIB_PATH} has ABI version {got}, this binding expects "
                           f"{ABI_VERSION}: rebuild it with __graft_entry__.build()")
    lib.discord_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.discord_default_opts.restype = None
    lib.discord_workspace_bytes.argtypes = [i64, i32, ctypes.POINTER(Opts)]
    lib.discord_workspace_bytes.restype = ctypes.c_size_t
    lib.discord_prepare.argtypes = [vp, i64, i32, ctypes.POINTER(Opts), vp, ctypes.c_size_t, vp,
                                    ctypes.POINTER(vp)]
    lib.discord_prepare.restype = ctypes.c_int
    lib.discord_search.argtypes = [vp, ctypes.POINTER(Result)]
    lib.discord_search.restype = ctypes.c_int
    lib.discord_search_graph.argtypes = [vp, ctypes.POINTER(Result)]
    lib.discord_search_graph.restype = ctypes.c_int
    lib.discord_release.argtypes = [vp]
    lib.discord_release.restype = None
    lib.discord_strerror.argtypes = [ctypes.c_int]
    lib.discord_strerror.restype = ctypes.c_char_p
    lib.discord_plan_error.argtypes = [vp]
    lib.discord_plan_error.restype = ctypes.c_char_p
    lib.discord_sax_breakpoints.argtypes = [i32, ctypes.POINTER(ctypes.c_double)]
    lib.discord_sax_breakpoints.restype = ctypes.c_int
    lib.discord_search_series.argtypes = [vp, i64, i32, ctypes.POINTER(i64),
                                          ctypes.POINTER(ctypes.c_double)]
    lib.discord_search_series.restype = ctypes.c_int
    lib.discord_search_series_noalloc.argtypes = [vp, i64, i32, ctypes.POINTER(Opts), vp,
                                                  ctypes.POINTER(Result)]
    lib.discord_search_series_noalloc.restype = ctypes.c_int
    lib.discord_search_once.argtypes = [vp, i64, i32, ctypes.POINTER(Opts), vp, ctypes.c_size_t,
                                        vp, ctypes.POINTER(Result)]
    lib.discord_search_once.restype = ctypes.c_int
    lib.discord_plan_count.argtypes = [vp, i32]
    lib.discord_plan_count.restype = i64
    lib.discord_plan_copy.argtypes = [vp, i32, vp, ctypes.c_size_t]
    lib.discord_plan_copy.restype = ctypes.c_int
    lib.discord_rows_nn_fp64.argtypes = [vp, vp, i64, vp, vp]
    lib.discord_rows_nn_fp64.restype = ctypes.c_int
    lib.discord_cu_mask.argtypes = [i32, i32, i32, ctypes.POINTER(ctypes.c_uint32), i32]
    lib.discord_cu_mask.restype = ctypes.c_int
    lib.discord_stream_create_cu_limited.argtypes = [i32, ctypes.POINTER(vp)]
    lib.discord_stream_create_cu_limited.restype = ctypes.c_int
    lib.discord_stream_destroy.argtypes = [vp]
    lib.discord_stream_destroy.restype = ctypes.c_int
    lib.discord_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    lib.discord_server_create.restype = ctypes.c_int
    lib.discord_server_create_with_executor.argtypes = [ctypes.POINTER(ServerConfig), EXECUTOR_FN,
                                                        vp, ctypes.POINTER(vp)]
    lib.discord_server_create_with_executor.restype = ctypes.c_int
    lib.discord_server_submit.argtypes = [vp, vp, i64, i32, ctypes.c_uint64]
    lib.discord_server_submit.restype = ctypes.c_int
    lib.discord_server_poll.argtypes = [vp, ctypes.POINTER(Completion), i32, i32,
                                        ctypes.POINTER(i32)]
    lib.discord_server_poll.restype = ctypes.c_int
    lib.discord_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.discord_server_get_stats.restype = ctypes.c_int
    lib.discord_server_destroy.argtypes = [vp]
    lib.discord_server_destroy.restype = None
    _lib = lib
    return lib


def strerror(status: int) -> str:
    return load().discord_strerror(status).decode()


def _check(status: int, plan=None):
    if status != 0:
        detail = load().discord_plan_error(plan).decode() if plan is not None else ""
        raise DiscordError(status, strerror(status) + (f": {detail}" if detail else ""))


def default_opts(**kw) -> Opts:
    o = Opts()
    load().discord_default_opts(ctypes.byref(o))
    if "precision" in kw:
        kw["precision"] = _PREC[kw["precision"]]
    for k, v in kw.items():
        if v is not None:
            setattr(o, k, int(v))
    return o


def workspace_bytes(m: int, n: int, **kw) -> int:
    o = default_opts(**kw)
    return int(load().discord_workspace_bytes(m, n, ctypes.byref(o)))


def sax_breakpoints(alpha: int) -> np.ndarray:
    out = (ctypes.c_double * max(alpha - 1, 1))()
    _check(load().discord_sax_breakpoints(alpha, out))
    return np.array(out[:alpha - 1], dtype=np.float64)


def _series_ptr(T):
    """(pointer, m, keepalive, stream) for a numpy array or a torch tensor."""
    try:
        import torch
        if isinstance(T, torch.Tensor):
            if T.dtype != torch.float32 or T.dim() != 1:
                raise ValueError("series must be a 1-D float32 tensor")
            t = T.contiguous()
            stream = torch.cuda.current_stream(t.device).cuda_stream if t.is_cuda else None
            return t.data_ptr(), t.numel(), t, stream
    except ImportError:
        pass
    a = np.ascontiguousarray(T, dtype=np.float32)
    if a.ndim != 1:
        raise ValueError("series must be one-dimensional")
    return a.ctypes.data, a.size, a, None


def cu_mask(total_cus: int, xccs: int, cus: int) -> list:
    """The CU mask of a stream limited to `cus` CUs (discord_cu_mask), as 32-bit
    words; host only."""
    lib = load()
    nw = (total_cus + 31) // 32
    buf = (ctypes.c_uint32 * max(nw, 1))()
    got = lib.discord_cu_mask(total_cus, xccs, cus, buf, nw)
    _check(got if got < 0 else 0)
    return list(buf[:got])


class CULimitedStream:
    """A HIP stream whose kernels run on `cus` compute units of the current
    device only (discord_stream_create_cu_limited); pass it as `stream=`.
    `handle` is the hipStream_t."""

    def __init__(self, cus: int):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.discord_stream_create_cu_limited(int(cus), ctypes.byref(h)))
        self.cus = int(cus)
        self.handle = h.value

    def close(self):
        if self.handle:
            h, self.handle = self.handle, None
            _check(load().discord_stream_destroy(h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Plan:
    """A prepared series (discord_prepare) that can be searched repeatedly."""

    def __init__(self, T, n: int, precision="fp32", abandon=True, order=2,
                 paa_w=4, alphabet=4, probe_steps=0, znorm=False, stream=None,
                 torch_workspace=False):
        lib = load()
        self.opts = default_opts(precision=precision, abandon=int(bool(abandon)),
                                 order=int(order), paa_w=paa_w,
                                 alphabet=alphabet, probe_steps=probe_steps,
                                 znorm=int(bool(znorm)))
        ptr, m, self._keep, tstream = _series_ptr(T)
        self.m, self.n = int(m), int(n)
        self.N = self.m - self.n + 1
        if stream is None:
            stream = tstream
        elif hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        elif isinstance(stream, CULimitedStream):
            stream = stream.handle
        self._ws = None
        ws_ptr, ws_bytes = None, 0
        if torch_workspace:
            import torch
            ws_bytes = lib.discord_workspace_bytes(self.m, self.n, ctypes.byref(self.opts))
            if ws_bytes == 0:
                _check(-1)
            self._ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device="cuda")
            base = self._ws.data_ptr()
            ws_ptr = (base + 255) // 256 * 256
        h = ctypes.c_void_p()
        st = lib.discord_prepare(ctypes.c_void_p(ptr), self.m, self.n, ctypes.byref(self.opts),
                                 ws_ptr, ws_bytes, stream, ctypes.byref(h))
        if st != 0:
            detail = lib.discord_plan_error(None).decode()
            raise DiscordError(st, strerror(st) + (f": {detail}" if detail else ""))
        self._h = h

    def search(self) -> Result:
        r = Result()
        _check(load().discord_search(self._h, ctypes.byref(r)), self._h)
        return r

    def search_graph(self) -> Result:
        """discord_search_graph: captured into a HIP graph on the first call,
        replayed afterwards."""
        r = Result()
        _check(load().discord_search_graph(self._h, ctypes.byref(r)), self._h)
        return r

    def count(self, field: str) -> int:
        c = load().discord_plan_count(self._h, FIELD[field][0])
        if c < 0:
            _check(int(c), self._h)
        return int(c)

    def copy(self, field: str) -> np.ndarray:
        code, dt = FIELD[field]
        c = self.count(field)
        out = np.empty(c, dtype=dt)
        _check(load().discord_plan_copy(self._h, code, out.ctypes.data, out.nbytes), self._h)
        return out

    def rows_nn_fp64(self, rows):
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        d = np.empty(rows.size, dtype=np.float64)
        j = np.empty(rows.size, dtype=np.int64)
        _check(load().discord_rows_nn_fp64(self._h, rows.ctypes.data, rows.size, d.ctypes.data,
                                           j.ctypes.data), self._h)
        return d, j

    def release(self):
        if getattr(self, "_h", None):
            load().discord_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.release()


def search_once(T, n: int, precision="fp32", stream=None, torch_workspace=True,
                **opts) -> Result:
    """discord_search_once: preparation and search of one series as one device
    sequence with one synchronisation.  torch_workspace: the workspace is a
    torch tensor (from torch's caching allocator); else the library allocates
    and frees one per call."""
    lib = load()
    o = default_opts(precision=precision, **opts)
    ptr, m, keep, tstream = _series_ptr(T)
    if stream is None:
        stream = tstream
    elif hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    elif isinstance(stream, CULimitedStream):
        stream = stream.handle
    ws, ws_ptr, ws_bytes = None, None, 0
    if torch_workspace:
        import torch
        ws_bytes = lib.discord_workspace_bytes(m, n, ctypes.byref(o))
        if ws_bytes == 0:
            _check(-1)
        ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device="cuda")
        ws_ptr = (ws.data_ptr() + 255) // 256 * 256
    r = Result()
    st = lib.discord_search_once(ctypes.c_void_p(ptr), m, n, ctypes.byref(o), ws_ptr, ws_bytes,
                                 stream, ctypes.byref(r))
    del ws   # the call has synchronised its stream
    if st != 0:
        detail = lib.discord_plan_error(None).decode()
        raise DiscordError(st, strerror(st) + (f": {detail}" if detail else ""))
    return r


def search(T, n: int, precision="fp32", **kw):
    """One search of one series (discord_search_once): returns (index,
    distance, result-dict)."""
    r = search_once(T, n, precision=precision, **kw)
    return int(r.index), float(r.distance), r.as_dict()


def search_series(T, n: int):
    ptr, m, keep, _ = _series_ptr(T)
    idx = ctypes.c_int64()
    dist = ctypes.c_double()
    _check(load().discord_search_series(ctypes.c_void_p(ptr), m, n, ctypes.byref(idx),
                                        ctypes.byref(dist)))
    return int(idx.value), float(dist.value)


def search_series_noalloc(T, n: int, stream=None, **opts) -> Result:
    """discord_search_series_noalloc: prepare + search in the library's static
    device workspace (no allocation; plans up to NOALLOC_MAX_BYTES)."""
    ptr, m, keep, tstream = _series_ptr(T)
    if stream is None:
        stream = tstream
    elif hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    elif isinstance(stream, CULimitedStream):
        stream = stream.handle
    o = default_opts(**opts)
    r = Result()
    st = load().discord_search_series_noalloc(ctypes.c_void_p(ptr), m, n, ctypes.byref(o),
                                              ctypes.c_void_p(stream), ctypes.byref(r))
    if st != 0:
        detail = load().discord_plan_error(None).decode()
        raise DiscordError(st, strerror(st) + (f": {detail}" if detail else ""))
    return r


class Server:
    """The serving loop (discord_server_*): FIFO admission by slot and HBM
    footprint, one worker stream per slot, completions polled by the caller.

    `executor`: None for the GPU path; else a Python callable
    ``executor(request: Request, opts: Opts, result: Result) -> int`` run on a
    worker thread with a virtual arena (for cost models and host tests)."""

    def __init__(self, budget_bytes: int, slots: int = 4, max_queued: int = 0,
                 executor=None, **opts):
        lib = load()
        self.cfg = ServerConfig(int(budget_bytes), int(slots), int(max_queued),
                                default_opts(**opts))
        h = ctypes.c_void_p()
        if executor is None:
            self._fn = None
            st = lib.discord_server_create(ctypes.byref(self.cfg), ctypes.byref(h))
        else:
            def trampoline(ctx, req, o, res, detail, detail_len):
                try:
                    return int(executor(req.contents, o.contents, res.contents))
                except Exception as e:  # an executor error becomes the request's status
                    msg = f"{type(e).__name__}: {e}".encode()[:max(int(detail_len) - 1, 0)]
                    if detail and detail_len:
                        ctypes.memmove(detail, msg + b"\0", len(msg) + 1)
                    return -4
            self._fn = EXECUTOR_FN(trampoline)
            st = lib.discord_server_create_with_executor(ctypes.byref(self.cfg), self._fn, None,
                                                         ctypes.byref(h))
        _check(st)
        self._h = h

    def submit(self, T, n: int, tag: int) -> int:
        """Queue a request (host float32 series); returns the status (0 = queued)."""
        a = np.ascontiguousarray(T, dtype=np.float32)
        if a.ndim != 1:
            raise ValueError("series must be one-dimensional")
        return int(load().discord_server_submit(self._h, ctypes.c_void_p(a.ctypes.data), a.size,
                                                int(n), int(tag)))

    def poll(self, max_count: int = 64, timeout_ms: int = 0) -> list:
        buf = (Completion * max_count)()
        cnt = ctypes.c_int32()
        _check(load().discord_server_poll(self._h, buf, max_count, int(timeout_ms),
                                          ctypes.byref(cnt)))
        return [buf[i].as_dict() for i in range(cnt.value)]

    def stats(self) -> dict:
        s = ServerStats()
        _check(load().discord_server_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            load().discord_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
