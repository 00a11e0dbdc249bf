"""Python binding of ``include/hj.h`` (ctypes; argument marshalling only).

Every function here forwards to ``libhj.so``; no step of the join runs in
Python and there is no fallback: if the library is missing, loading fails
loudly.  PyTorch supplies device memory and streams.  ``torch`` is imported
before the library is loaded so that the library binds to the HIP runtime
torch already loaded (one runtime per process).
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhj.so")

HJ_OK = 0
HJ_ERR_INVALID = 1
HJ_ERR_CAPACITY = 2
HJ_ERR_WORKSPACE = 3
HJ_ERR_DEVICE = 4
HJ_ERR_UNSUPPORTED = 5

HJ_SHJ = 0
HJ_PHJ = 1
HJ_AUTO = 2
HJ_HASH_IDENTITY = 0
HJ_HASH_MURMUR2 = 1
HJ_FLAG_ONE_PASS = 1

HJ_BATCH_NO_GRAPH = 1

# Every symbol include/hj.h declares.
EXPORTED = (
    "hj_default_params", "hj_resolve_params", "hj_workspace_bytes", "hj_join", "hj_join_sync", "hj_join_timed",
    "hj_join_noalloc", "hj_join_external", "hj_model_seconds",
    "hj_batch_plan_create", "hj_batch_workspace_bytes", "hj_batch_direct_jobs", "hj_batch_graph_nodes", "hj_batch_run",
    "hj_batch_plan_destroy", "hj_batch_bytes", "hj_batch", "hj_table_bytes", "hj_build",
    "hj_probe_workspace_bytes", "hj_probe", "hj_server_create", "hj_server_submit", "hj_server_submit_probe", "hj_server_poll", "hj_server_drain",
    "hj_server_stats", "hj_server_destroy", "hj_workspace_status", "hj_status_str", "hj_last_error",
    "hj_version",
)


class HjRel(ctypes.Structure):
    _fields_ = [("key", ctypes.c_void_p), ("rid", ctypes.c_void_p), ("n", ctypes.c_uint64)]


class HjOut(ctypes.Structure):
    _fields_ = [("rid_r", ctypes.c_void_p), ("rid_s", ctypes.c_void_p), ("capacity", ctypes.c_uint64)]


class HjParams(ctypes.Structure):
    _fields_ = [
        ("algo", ctypes.c_uint32), ("passes", ctypes.c_uint32), ("bits", ctypes.c_uint32 * 2),
        ("hash", ctypes.c_uint32), ("tile", ctypes.c_uint32), ("lds_cap", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
    ]

    def __repr__(self) -> str:
        return ("HjParams(algo=%s, passes=%d, bits=(%d, %d), hash=%d, tile=%d, lds_cap=%d, flags=%d)" % (
            {HJ_SHJ: "shj", HJ_PHJ: "phj", HJ_AUTO: "auto"}.get(self.algo, str(self.algo)), self.passes,
            self.bits[0], self.bits[1], self.hash, self.tile, self.lds_cap, self.flags))


class HjTable(ctypes.Structure):
    _fields_ = [("params", HjParams), ("n_r", ctypes.c_uint64), ("r_key", ctypes.c_void_p),
                ("r_rid", ctypes.c_void_p), ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t)]


class HjJob(ctypes.Structure):
    _fields_ = [("R", HjRel), ("S", HjRel), ("out", HjOut), ("d_count", ctypes.c_void_p)]


class HjServerConfig(ctypes.Structure):
    _fields_ = [("mem_cap_bytes", ctypes.c_uint64), ("slots", ctypes.c_uint32),
                ("max_batch_jobs", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class HjExternalInfo(ctypes.Structure):
    _fields_ = [("fanout_bits", ctypes.c_uint32), ("pieces", ctypes.c_uint32), ("chunk_tuples", ctypes.c_uint64),
                ("partition_s", ctypes.c_double), ("join_s", ctypes.c_double), ("total_s", ctypes.c_double),
                ("h2d_bytes", ctypes.c_uint64), ("d2h_bytes", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class HJError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s (status %d): %s" % (_status_name(status), status, message))
        self.status = status
        self.message = message


_lock = threading.Lock()
_lib = None


def load() -> ctypes.CDLL:
    """Loads ``libhj.so`` (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise FileNotFoundError(
                    "%s is missing: build it with `python -m paper_1307_1955_amd.build`" % LIB_PATH)
            lib = ctypes.CDLL(LIB_PATH)
            P = ctypes.POINTER
            vp = ctypes.c_void_p
            lib.hj_default_params.restype = None
            lib.hj_default_params.argtypes = [P(HjParams)]
            lib.hj_resolve_params.restype = ctypes.c_int
            lib.hj_resolve_params.argtypes = [P(HjParams), ctypes.c_uint64, ctypes.c_uint64, P(HjParams)]
            lib.hj_workspace_bytes.restype = ctypes.c_size_t
            lib.hj_workspace_bytes.argtypes = [P(HjParams), ctypes.c_uint64, ctypes.c_uint64]
            lib.hj_join.restype = ctypes.c_int
            lib.hj_join.argtypes = [P(HjParams), P(HjRel), P(HjRel), P(HjOut), vp, ctypes.c_size_t, vp, vp]
            lib.hj_join_sync.restype = ctypes.c_int
            lib.hj_join_sync.argtypes = [P(HjParams), P(HjRel), P(HjRel), P(HjOut), vp, ctypes.c_size_t, vp,
                                         P(ctypes.c_uint64), vp]
            lib.hj_join_timed.restype = ctypes.c_int
            lib.hj_join_timed.argtypes = [P(HjParams), P(HjRel), P(HjRel), P(HjOut), vp, ctypes.c_size_t, vp,
                                          vp, P(ctypes.c_char_p), P(ctypes.c_float), ctypes.c_uint32,
                                          P(ctypes.c_uint32)]
            lib.hj_join_noalloc.restype = ctypes.c_int
            lib.hj_join_noalloc.argtypes = [P(HjParams), P(HjRel), P(HjRel), P(HjOut), vp, vp]
            lib.hj_model_seconds.restype = ctypes.c_int
            lib.hj_model_seconds.argtypes = [P(HjParams), ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                             P(ctypes.c_double)]
            lib.hj_join_external.restype = ctypes.c_int
            lib.hj_join_external.argtypes = [P(HjParams), P(HjRel), P(HjRel), P(HjOut), vp, ctypes.c_size_t,
                                             P(ctypes.c_uint64), P(HjExternalInfo)]
            lib.hj_table_bytes.restype = ctypes.c_size_t
            lib.hj_table_bytes.argtypes = [P(HjParams), ctypes.c_uint64]
            lib.hj_build.restype = ctypes.c_int
            lib.hj_build.argtypes = [P(HjParams), P(HjRel), vp, ctypes.c_size_t, vp, P(HjTable)]
            lib.hj_probe_workspace_bytes.restype = ctypes.c_size_t
            lib.hj_probe_workspace_bytes.argtypes = [P(HjTable), ctypes.c_uint64]
            lib.hj_probe.restype = ctypes.c_int
            lib.hj_probe.argtypes = [P(HjTable), P(HjRel), P(HjOut), vp, ctypes.c_size_t, vp, vp]
            lib.hj_batch_bytes.restype = ctypes.c_size_t
            lib.hj_batch_bytes.argtypes = [ctypes.c_uint32, P(HjJob), P(HjParams)]
            lib.hj_batch.restype = ctypes.c_int
            lib.hj_batch.argtypes = [ctypes.c_uint32, P(HjJob), P(HjParams), vp, ctypes.c_size_t, vp]
            lib.hj_workspace_status.restype = ctypes.c_int
            lib.hj_workspace_status.argtypes = [vp, vp]
            lib.hj_status_str.restype = ctypes.c_char_p
            lib.hj_status_str.argtypes = [ctypes.c_int]
            lib.hj_last_error.restype = ctypes.c_char_p
            lib.hj_last_error.argtypes = []
            lib.hj_version.restype = ctypes.c_uint32
            lib.hj_version.argtypes = []
            lib.hj_batch_plan_create.restype = ctypes.c_int
            lib.hj_batch_plan_create.argtypes = [ctypes.c_uint32, P(HjJob), P(HjParams), ctypes.c_uint32,
                                                 P(ctypes.c_void_p)]
            lib.hj_batch_workspace_bytes.restype = ctypes.c_size_t
            lib.hj_batch_workspace_bytes.argtypes = [ctypes.c_void_p]
            lib.hj_batch_direct_jobs.restype = ctypes.c_uint32
            lib.hj_batch_direct_jobs.argtypes = [ctypes.c_void_p]
            lib.hj_batch_graph_nodes.restype = ctypes.c_size_t
            lib.hj_batch_graph_nodes.argtypes = [ctypes.c_void_p]
            lib.hj_batch_run.restype = ctypes.c_int
            lib.hj_batch_run.argtypes = [ctypes.c_void_p, vp, ctypes.c_size_t, vp]
            lib.hj_batch_plan_destroy.restype = None
            lib.hj_batch_plan_destroy.argtypes = [ctypes.c_void_p]
            lib.hj_server_create.restype = ctypes.c_int
            lib.hj_server_create.argtypes = [P(HjServerConfig), vp, ctypes.c_size_t, P(ctypes.c_void_p)]
            lib.hj_server_submit.restype = ctypes.c_int
            lib.hj_server_submit.argtypes = [ctypes.c_void_p, P(HjJob), P(HjParams), ctypes.c_uint64,
                                             P(ctypes.c_uint64)]
            lib.hj_server_submit_probe.restype = ctypes.c_int
            lib.hj_server_submit_probe.argtypes = [ctypes.c_void_p, P(HjTable), P(HjRel), P(HjOut), vp,
                                                   ctypes.c_uint64, P(ctypes.c_uint64)]
            lib.hj_server_poll.restype = ctypes.c_int
            lib.hj_server_poll.argtypes = [ctypes.c_void_p, P(ctypes.c_uint64), P(ctypes.c_int32),
                                           P(ctypes.c_double), P(ctypes.c_double), ctypes.c_uint32,
                                           P(ctypes.c_uint32)]
            lib.hj_server_drain.restype = ctypes.c_int
            lib.hj_server_drain.argtypes = [ctypes.c_void_p]
            lib.hj_server_stats.restype = ctypes.c_int
            lib.hj_server_stats.argtypes = [ctypes.c_void_p] + [P(ctypes.c_uint64)] * 4
            lib.hj_server_destroy.restype = None
            lib.hj_server_destroy.argtypes = [ctypes.c_void_p]
            _lib = lib
    return _lib


def _status_name(s: int) -> str:
    try:
        return load().hj_status_str(s).decode()
    except Exception:
        return "status"


def _check(status: int) -> None:
    if status != HJ_OK:
        raise HJError(status, load().hj_last_error().decode())


def hj_default_params() -> HjParams:
    p = HjParams()
    load().hj_default_params(ctypes.byref(p))
    return p


def params(algo: str = "phj", passes: int = 2, bits=(6, 6), hash: str = "identity", tile: int = 0,
           lds_cap: int = 0, one_pass: bool = False) -> HjParams:
    """Builds an ``hj_params``.  ``algo`` is "shj", "phj" or "auto"; ``hash`` "identity" or "murmur2";
    ``one_pass`` selects the single-pass PHJ output (HJ_FLAG_ONE_PASS)."""
    p = HjParams()
    p.algo = {"shj": HJ_SHJ, "phj": HJ_PHJ, "auto": HJ_AUTO}[algo]
    p.passes = passes
    b = tuple(bits) + (0,) * (2 - len(tuple(bits)))
    p.bits[0], p.bits[1] = int(b[0]), int(b[1])
    p.hash = {"identity": HJ_HASH_IDENTITY, "murmur2": HJ_HASH_MURMUR2}[hash]
    p.tile = tile
    p.lds_cap = lds_cap
    p.flags = HJ_FLAG_ONE_PASS if one_pass else 0
    return p


def hj_resolve_params(p: HjParams, n_r: int, n_s: int) -> HjParams:
    """The parameters as hj_join uses them for these sizes (tile, lds_cap filled in)."""
    q = HjParams()
    _check(load().hj_resolve_params(ctypes.byref(p), n_r, n_s, ctypes.byref(q)))
    return q


def hj_model_seconds(p: HjParams, n_r: int, n_s: int, pairs: int) -> float:
    """The library's cost-model prediction of hj_join's time (seconds)."""
    v = ctypes.c_double(0.0)
    _check(load().hj_model_seconds(ctypes.byref(p), n_r, n_s, pairs, ctypes.byref(v)))
    return float(v.value)


def hj_workspace_bytes(p: HjParams, n_r: int, n_s: int) -> int:
    v = load().hj_workspace_bytes(ctypes.byref(p), n_r, n_s)
    if v == 0:
        raise HJError(HJ_ERR_INVALID, load().hj_last_error().decode())
    return int(v)


def hj_workspace_status(ws: torch.Tensor, stream=None) -> None:
    """Synchronises ``stream`` and raises ``HJError`` (HJ_ERR_DEVICE) when the
    error word of the workspace ``ws`` (the last call that used it) is set."""
    wp, _ = _ws(ws)
    _check(load().hj_workspace_status(wp, _stream(stream)))


def hj_version() -> int:
    return int(load().hj_version())


def _dev_i32(t: torch.Tensor, name: str) -> int:
    if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous() or t.dim() != 1:
        raise ValueError("%s must be a contiguous 1-D int32 CUDA tensor" % name)
    return t.data_ptr()


def _rel(key: torch.Tensor, rid: torch.Tensor, name: str) -> HjRel:
    if key.numel() != rid.numel():
        raise ValueError("%s: key and rid lengths differ" % name)
    return HjRel(_dev_i32(key, name + ".key"), _dev_i32(rid, name + ".rid"), key.numel())


def _out(out_r: torch.Tensor, out_s: torch.Tensor) -> HjOut:
    if out_r.numel() != out_s.numel():
        raise ValueError("output columns differ in length")
    return HjOut(_dev_i32(out_r, "out_r"), _dev_i32(out_s, "out_s"), out_r.numel())


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _ws(ws: torch.Tensor) -> tuple[int, int]:
    if not ws.is_cuda or not ws.is_contiguous():
        raise ValueError("workspace must be a contiguous CUDA tensor")
    return ws.data_ptr(), ws.numel() * ws.element_size()


def workspace(p: HjParams, n_r: int, n_s: int, device="cuda") -> torch.Tensor:
    """A device workspace tensor of the size hj_workspace_bytes asks for."""
    nbytes = hj_workspace_bytes(p, n_r, n_s)
    # torch's allocator returns 512-byte aligned blocks
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def hj_join(p: HjParams, r_key, r_rid, s_key, s_rid, out_r, out_s, ws: torch.Tensor,
            d_count: torch.Tensor, stream=None) -> None:
    """Enqueues the join on ``stream`` (torch's current stream by default)."""
    if d_count.dtype != torch.int64 or not d_count.is_cuda or d_count.numel() < 1:
        raise ValueError("d_count must be an int64 CUDA tensor with at least one element")
    R, S, O = _rel(r_key, r_rid, "R"), _rel(s_key, s_rid, "S"), _out(out_r, out_s)
    wp, wb = _ws(ws)
    _check(load().hj_join(ctypes.byref(p), ctypes.byref(R), ctypes.byref(S), ctypes.byref(O), wp, wb,
                          d_count.data_ptr(), _stream(stream)))


def hj_join_sync(p: HjParams, r_key, r_rid, s_key, s_rid, out_r, out_s, ws: torch.Tensor,
                 d_count: torch.Tensor, stream=None, raise_on_capacity: bool = True) -> int:
    """Joins, synchronises the stream and returns the number of pairs."""
    if d_count.dtype != torch.int64 or not d_count.is_cuda or d_count.numel() < 1:
        raise ValueError("d_count must be an int64 CUDA tensor with at least one element")
    R, S, O = _rel(r_key, r_rid, "R"), _rel(s_key, s_rid, "S"), _out(out_r, out_s)
    wp, wb = _ws(ws)
    h = ctypes.c_uint64(0)
    st = load().hj_join_sync(ctypes.byref(p), ctypes.byref(R), ctypes.byref(S), ctypes.byref(O), wp, wb,
                             d_count.data_ptr(), ctypes.byref(h), _stream(stream))
    if st == HJ_ERR_CAPACITY and not raise_on_capacity:
        return int(h.value)
    _check(st)
    return int(h.value)


def hj_join_timed(p: HjParams, r_key, r_rid, s_key, s_rid, out_r, out_s, ws: torch.Tensor,
                  d_count: torch.Tensor, stream=None, max_launches: int = 64) -> list[tuple[str, float]]:
    """One join with every launch bracketed by HIP events; returns (kernel, ms) per launch."""
    R, S, O = _rel(r_key, r_rid, "R"), _rel(s_key, s_rid, "S"), _out(out_r, out_s)
    wp, wb = _ws(ws)
    names = (ctypes.c_char_p * max_launches)()
    ms = (ctypes.c_float * max_launches)()
    n = ctypes.c_uint32(0)
    _check(load().hj_join_timed(ctypes.byref(p), ctypes.byref(R), ctypes.byref(S), ctypes.byref(O), wp, wb,
                                d_count.data_ptr(), _stream(stream), names, ms, max_launches,
                                ctypes.byref(n)))
    return [(names[i].decode(), float(ms[i])) for i in range(min(n.value, max_launches))]


def hj_join_noalloc(p: HjParams, r_key, r_rid, s_key, s_rid, out_r, out_s, d_count: torch.Tensor,
                    stream=None) -> None:
    """Enqueues the join on the library's fixed device workspace (no workspace
    argument, nothing allocated; see include/hj.h for its size limit)."""
    if d_count.dtype != torch.int64 or not d_count.is_cuda or d_count.numel() < 1:
        raise ValueError("d_count must be an int64 CUDA tensor with at least one element")
    R, S, O = _rel(r_key, r_rid, "R"), _rel(s_key, s_rid, "S"), _out(out_r, out_s)
    _check(load().hj_join_noalloc(ctypes.byref(p), ctypes.byref(R), ctypes.byref(S), ctypes.byref(O),
                                  d_count.data_ptr(), _stream(stream)))


def join(r_key, r_rid, s_key, s_rid, p: HjParams | None = None, capacity: int | None = None,
         stream=None):
    """Convenience: allocates workspace and output, joins, and returns
    ``(rid_r, rid_s, count)`` as CUDA tensors trimmed to ``count``.

    The output is first sized to ``capacity`` (default ``len(S)``, exact when
    R's keys are unique); if the join has more pairs it is rerun once with an
    output of the exact size."""
    if p is None:
        p = hj_default_params()
    dev = r_key.device
    ws = workspace(p, r_key.numel(), s_key.numel(), dev)
    d_count = torch.zeros(1, dtype=torch.int64, device=dev)
    cap = s_key.numel() if capacity is None else int(capacity)
    out_r = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    out_s = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    cnt = hj_join_sync(p, r_key, r_rid, s_key, s_rid, out_r[:cap], out_s[:cap], ws, d_count, stream,
                       raise_on_capacity=False)
    if cnt > cap:
        out_r = torch.empty(cnt, dtype=torch.int32, device=dev)
        out_s = torch.empty(cnt, dtype=torch.int32, device=dev)
        cnt2 = hj_join_sync(p, r_key, r_rid, s_key, s_rid, out_r, out_s, ws, d_count, stream)
        assert cnt2 == cnt
    return out_r[:cnt], out_s[:cnt], cnt


def _host_i32(a, name: str) -> int:
    """Address of a host int32 array: a contiguous CPU torch tensor (pinned or
    not) or a numpy array."""
    if isinstance(a, torch.Tensor):
        if a.dtype != torch.int32 or a.is_cuda or not a.is_contiguous() or a.dim() != 1:
            raise ValueError("%s must be a contiguous 1-D int32 CPU tensor" % name)
        return a.data_ptr()
    import numpy as np
    if not isinstance(a, np.ndarray) or a.dtype != np.int32 or not a.flags.c_contiguous or a.ndim != 1:
        raise ValueError("%s must be a contiguous 1-D int32 array" % name)
    return a.ctypes.data


def hj_join_external(p: HjParams, r_key, r_rid, s_key, s_rid, out_r, out_s, ws: torch.Tensor):
    """Joins relations held in HOST memory through the device workspace ``ws``
    (see include/hj.h); the pairs land in the host arrays ``out_r``/``out_s``.
    Returns ``(count, info)``; raises on errors, also when the count exceeds the
    output length (HJ_ERR_CAPACITY; the count is in the exception's message)."""
    if len(r_key) != len(r_rid) or len(s_key) != len(s_rid) or len(out_r) != len(out_s):
        raise ValueError("column lengths differ")
    R = HjRel(_host_i32(r_key, "r_key"), _host_i32(r_rid, "r_rid"), len(r_key))
    S = HjRel(_host_i32(s_key, "s_key"), _host_i32(s_rid, "s_rid"), len(s_key))
    O = HjOut(_host_i32(out_r, "out_r"), _host_i32(out_s, "out_s"), len(out_r))
    wp, wb = _ws(ws)
    h = ctypes.c_uint64(0)
    info = HjExternalInfo()
    _check(load().hj_join_external(ctypes.byref(p), ctypes.byref(R), ctypes.byref(S), ctypes.byref(O), wp, wb,
                                   ctypes.byref(h), ctypes.byref(info)))
    return int(h.value), info.as_dict()


# ---------------------------------------------------------------------------
# Build once, probe many times
# ---------------------------------------------------------------------------


def hj_table_bytes(p: HjParams, n_r: int) -> int:
    v = load().hj_table_bytes(ctypes.byref(p), n_r)
    if v == 0:
        raise HJError(HJ_ERR_INVALID, load().hj_last_error().decode())
    return int(v)


def hj_build(p: HjParams, r_key, r_rid, ws: torch.Tensor, stream=None) -> HjTable:
    """Enqueues the build of R's table into ``ws``; returns the ``hj_table``."""
    R = _rel(r_key, r_rid, "R")
    wp, wb = _ws(ws)
    t = HjTable()
    _check(load().hj_build(ctypes.byref(p), ctypes.byref(R), wp, wb, _stream(stream), ctypes.byref(t)))
    return t


def hj_probe_workspace_bytes(t: HjTable, n_s: int) -> int:
    v = load().hj_probe_workspace_bytes(ctypes.byref(t), n_s)
    if v == 0:
        raise HJError(HJ_ERR_INVALID, load().hj_last_error().decode())
    return int(v)


def hj_probe(t: HjTable, s_key, s_rid, out_r, out_s, ws: torch.Tensor, d_count: torch.Tensor,
             stream=None) -> None:
    """Enqueues a probe of table ``t`` by S on ``stream``."""
    if d_count.dtype != torch.int64 or not d_count.is_cuda or d_count.numel() < 1:
        raise ValueError("d_count must be an int64 CUDA tensor with at least one element")
    S, O = _rel(s_key, s_rid, "S"), _out(out_r, out_s)
    wp, wb = _ws(ws)
    _check(load().hj_probe(ctypes.byref(t), ctypes.byref(S), ctypes.byref(O), wp, wb, d_count.data_ptr(),
                           _stream(stream)))


class Table:
    """A table over R (``hj_build``) with its device workspace; keeps R's
    tensors alive for probes that read them.  ``probe`` joins S against it."""

    def __init__(self, r_key, r_rid, p: HjParams | None = None, stream=None):
        if p is None:
            p = hj_default_params()
        self.r_key, self.r_rid = r_key, r_rid
        self.ws = torch.empty(max(hj_table_bytes(p, r_key.numel()), 1), dtype=torch.uint8, device=r_key.device)
        self.t = hj_build(p, r_key, r_rid, self.ws, stream)

    @property
    def params(self) -> HjParams:
        return self.t.params

    def probe_workspace(self, n_s: int) -> torch.Tensor:
        return torch.empty(max(hj_probe_workspace_bytes(self.t, n_s), 1), dtype=torch.uint8,
                           device=self.r_key.device)

    def probe(self, s_key, s_rid, capacity: int | None = None, stream=None):
        """Returns ``(rid_r, rid_s, count)`` trimmed to ``count`` (rerun once with
        the exact size when ``capacity``, default ``len(S)``, is too small)."""
        dev = s_key.device
        ws = self.probe_workspace(s_key.numel())
        d_count = torch.zeros(1, dtype=torch.int64, device=dev)
        cap = s_key.numel() if capacity is None else int(capacity)
        for attempt in range(2):
            out_r = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            out_s = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            hj_probe(self.t, s_key, s_rid, out_r[:cap], out_s[:cap], ws, d_count, stream)
            (stream or torch.cuda.current_stream()).synchronize()
            cnt = int(d_count.item())
            if cnt <= cap:
                return out_r[:cnt], out_s[:cnt], cnt
            cap = cnt
        raise AssertionError("probe count changed between runs")


# ---------------------------------------------------------------------------
# Batches
# ---------------------------------------------------------------------------


def _job_array(jobs, d_counts: torch.Tensor, params):
    if d_counts.dtype != torch.int64 or not d_counts.is_cuda or d_counts.numel() < len(jobs):
        raise ValueError("d_counts must be an int64 CUDA tensor with one element per job")
    n = len(jobs)
    arr = (HjJob * max(n, 1))()
    base = d_counts.data_ptr()
    for j, (rk, rr, sk, sr, o_r, o_s) in enumerate(jobs):
        arr[j].R = _rel(rk, rr, "R")
        arr[j].S = _rel(sk, sr, "S")
        arr[j].out = _out(o_r, o_s)
        arr[j].d_count = base + 8 * j
    pp = None
    if params is not None:
        if len(params) != n:
            raise ValueError("one HjParams per job")
        pp = (HjParams * max(n, 1))(*params)
    return n, arr, pp


def hj_batch_bytes(jobs, d_counts: torch.Tensor, params=None) -> int:
    n, arr, pp = _job_array(jobs, d_counts, params)
    v = load().hj_batch_bytes(n, arr, pp)
    if v == 0:
        raise HJError(HJ_ERR_INVALID, load().hj_last_error().decode())
    return int(v)


def hj_batch(jobs, d_counts: torch.Tensor, ws: torch.Tensor, params=None, stream=None) -> None:
    """One-shot batch (``hj_batch``): plans, runs and synchronises ``stream``."""
    n, arr, pp = _job_array(jobs, d_counts, params)
    wp, wb = _ws(ws)
    _check(load().hj_batch(n, arr, pp, wp, wb, _stream(stream)))


class BatchPlan:
    """``hj_batch_plan`` over jobs given as tensors.

    jobs: sequence of (r_key, r_rid, s_key, s_rid, out_r, out_s) CUDA tensors;
    d_counts: int64 CUDA tensor with one element per job (job j's count is
    d_counts[j]); params: sequence of HjParams (one per job) or None for the
    library's choice per job (HJ_AUTO, one-pass); graph=False enqueues
    without a HIP graph.
    The tensors must stay alive while the plan is used."""

    def __init__(self, jobs, d_counts: torch.Tensor, params=None, graph: bool = True):
        n, arr, pp = _job_array(jobs, d_counts, params)
        self._keep = (jobs, d_counts)
        h = ctypes.c_void_p()
        _check(load().hj_batch_plan_create(n, arr, pp, 0 if graph else HJ_BATCH_NO_GRAPH, ctypes.byref(h)))
        self._h = h
        self.njobs = n

    @property
    def workspace_bytes(self) -> int:
        return int(load().hj_batch_workspace_bytes(self._h))

    @property
    def direct_jobs(self) -> int:
        return int(load().hj_batch_direct_jobs(self._h))

    @property
    def graph_nodes(self) -> int:
        """Nodes of the captured graph (0 before the first graph run)."""
        return int(load().hj_batch_graph_nodes(self._h))

    def workspace(self, device="cuda") -> torch.Tensor:
        return torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8, device=device)

    def run(self, ws: torch.Tensor, stream=None) -> None:
        wp, wb = _ws(ws)
        _check(load().hj_batch_run(self._h, wp, wb, _stream(stream)))

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().hj_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------


def make_job(r_key, r_rid, s_key, s_rid, out_r, out_s, d_count_ptr: int) -> HjJob:
    """An hj_job over tensors; d_count_ptr is the device address of its uint64 count."""
    j = HjJob()
    j.R = _rel(r_key, r_rid, "R")
    j.S = _rel(s_key, s_rid, "S")
    j.out = _out(out_r, out_s)
    j.d_count = d_count_ptr
    return j


class Server:
    """``hj_server``: continuous batching of join requests (see include/hj.h)."""

    def __init__(self, ws: torch.Tensor, mem_cap_bytes: int, slots: int = 4, max_batch_jobs: int = 64):
        cfg = HjServerConfig(mem_cap_bytes, slots, max_batch_jobs, 0)
        wp, wb = _ws(ws)
        h = ctypes.c_void_p()
        _check(load().hj_server_create(ctypes.byref(cfg), wp, wb, ctypes.byref(h)))
        self._h = h
        self._ws = ws
        self._keep = {}

    def submit_job(self, job: HjJob, params: HjParams, footprint: int, keep=None) -> int:
        """Queues a prepared HjJob; `keep` holds tensors alive until the request is polled."""
        t = ctypes.c_uint64(0)
        _check(load().hj_server_submit(self._h, ctypes.byref(job), ctypes.byref(params), footprint,
                                       ctypes.byref(t)))
        if keep is not None:
            self._keep[t.value] = keep
        return int(t.value)

    def submit(self, r_key, r_rid, s_key, s_rid, out_r, out_s, d_count: torch.Tensor, params: HjParams,
               footprint: int) -> int:
        job = make_job(r_key, r_rid, s_key, s_rid, out_r, out_s, d_count.data_ptr())
        return self.submit_job(job, params, footprint, keep=(r_key, r_rid, s_key, s_rid, out_r, out_s, d_count))

    def submit_probe(self, table: "Table", s_key, s_rid, out_r, out_s, d_count: torch.Tensor,
                     footprint: int) -> int:
        """Queues a probe of a resident ``Table`` by S; the table must outlive the request."""
        S, O = _rel(s_key, s_rid, "S"), _out(out_r, out_s)
        t = ctypes.c_uint64(0)
        _check(load().hj_server_submit_probe(self._h, ctypes.byref(table.t), ctypes.byref(S), ctypes.byref(O),
                                             d_count.data_ptr(), footprint, ctypes.byref(t)))
        self._keep[t.value] = (table, s_key, s_rid, out_r, out_s, d_count)
        return int(t.value)

    def poll(self, max_n: int = 4096):
        """Finished requests: list of (ticket, status, latency_s, queue_s)."""
        tk = (ctypes.c_uint64 * max_n)()
        st = (ctypes.c_int32 * max_n)()
        lat = (ctypes.c_double * max_n)()
        qu = (ctypes.c_double * max_n)()
        n = ctypes.c_uint32(0)
        _check(load().hj_server_poll(self._h, tk, st, lat, qu, max_n, ctypes.byref(n)))
        out = [(int(tk[i]), int(st[i]), float(lat[i]), float(qu[i])) for i in range(n.value)]
        for t, *_ in out:
            self._keep.pop(t, None)
        return out

    def drain(self) -> None:
        _check(load().hj_server_drain(self._h))

    def stats(self) -> dict:
        v = [ctypes.c_uint64(0) for _ in range(4)]
        _check(load().hj_server_stats(self._h, *[ctypes.byref(x) for x in v]))
        return {"completed": v[0].value, "rejected": v[1].value, "batches": v[2].value,
                "bytes_in_use": v[3].value}

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().hj_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
