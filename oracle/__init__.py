"""CPU oracle for the equi hash join -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never does, and shares no code with it.

``oracle.c`` is a plain single-threaded chained hash join written in the order
of the paper's Algorithm 1 (Section 3.1); see its header for the steps.  This
module compiles it on first use if ``liboracle.so`` is missing and wraps it
with numpy arrays.  ``canonical`` orders a pair multiset for comparison
(output order is unspecified by the method, so results are compared as
multisets).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = False) -> str:
    """Compiles ``oracle.c`` with gcc into ``liboracle.so``."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(LIB_PATH)
            lib.oracle_build.restype = ctypes.c_void_p
            lib.oracle_build.argtypes = [_i32p, _i32p, ctypes.c_uint64]
            lib.oracle_free.restype = None
            lib.oracle_free.argtypes = [ctypes.c_void_p]
            lib.oracle_probe_count.restype = ctypes.c_uint64
            lib.oracle_probe_count.argtypes = [ctypes.c_void_p, _i32p, ctypes.c_uint64]
            lib.oracle_probe_emit.restype = ctypes.c_uint64
            lib.oracle_probe_emit.argtypes = [ctypes.c_void_p, _i32p, _i32p, ctypes.c_uint64,
                                              _i32p, _i32p, ctypes.c_uint64]
            lib.oracle_nbuckets.restype = ctypes.c_uint64
            lib.oracle_nbuckets.argtypes = [ctypes.c_void_p]
            lib.oracle_nkeys.restype = ctypes.c_int64
            lib.oracle_nkeys.argtypes = [ctypes.c_void_p]
            lib.oracle_bucket_count.restype = ctypes.c_uint32
            lib.oracle_bucket_count.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
            lib.oracle_hash.restype = ctypes.c_uint32
            lib.oracle_hash.argtypes = [ctypes.c_int32]
            _lib = lib
    return _lib


def _arr(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_i32p)


class Table:
    """The paper's chained table built over R (steps b1-b4)."""

    def __init__(self, r_key, r_rid):
        self._lib = _load()
        self.r_key = _arr(r_key)
        self.r_rid = _arr(r_rid)
        if self.r_key.shape != self.r_rid.shape:
            raise ValueError("R key and rid lengths differ")
        self._h = self._lib.oracle_build(_ptr(self.r_key), _ptr(self.r_rid), len(self.r_key))
        if not self._h:
            raise MemoryError("oracle table allocation failed")

    def close(self):
        if self._h:
            self._lib.oracle_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def nbuckets(self) -> int:
        return int(self._lib.oracle_nbuckets(self._h))

    @property
    def nkeys(self) -> int:
        return int(self._lib.oracle_nkeys(self._h))

    def bucket_count(self, b: int) -> int:
        return int(self._lib.oracle_bucket_count(self._h, b))

    def probe_count(self, s_key) -> int:
        s_key = _arr(s_key)
        return int(self._lib.oracle_probe_count(self._h, _ptr(s_key), len(s_key)))

    def probe(self, s_key, s_rid) -> tuple[np.ndarray, np.ndarray]:
        """All (rid_R, rid_S) pairs in probe order (steps p1-p4)."""
        s_key = _arr(s_key)
        s_rid = _arr(s_rid)
        if s_key.shape != s_rid.shape:
            raise ValueError("S key and rid lengths differ")
        total = self.probe_count(s_key)
        out_r = np.empty(total, dtype=np.int32)
        out_s = np.empty(total, dtype=np.int32)
        got = int(self._lib.oracle_probe_emit(self._h, _ptr(s_key), _ptr(s_rid), len(s_key),
                                              _ptr(out_r), _ptr(out_s), total))
        assert got == total
        return out_r, out_s


    def probe_threads(self, s_key, s_rid, threads: int) -> tuple[np.ndarray, np.ndarray]:
        """``probe`` with S cut into ``threads`` contiguous chunks probed
        concurrently against the (read-only) table; the chunks' pairs are
        concatenated in chunk order, so the result equals ``probe``'s."""
        from concurrent.futures import ThreadPoolExecutor
        s_key = _arr(s_key)
        s_rid = _arr(s_rid)
        if s_key.shape != s_rid.shape:
            raise ValueError("S key and rid lengths differ")
        threads = max(1, int(threads))
        cuts = np.linspace(0, len(s_key), threads + 1).astype(np.int64)

        def chunk(i):  # the C calls release the interpreter lock
            k = np.ascontiguousarray(s_key[cuts[i]:cuts[i + 1]])
            r = np.ascontiguousarray(s_rid[cuts[i]:cuts[i + 1]])
            n = int(self._lib.oracle_probe_count(self._h, _ptr(k), len(k)))
            o_r = np.empty(n, dtype=np.int32)
            o_s = np.empty(n, dtype=np.int32)
            got = int(self._lib.oracle_probe_emit(self._h, _ptr(k), _ptr(r), len(k), _ptr(o_r), _ptr(o_s), n))
            assert got == n
            return o_r, o_s

        with ThreadPoolExecutor(max_workers=threads) as ex:
            parts = list(ex.map(chunk, range(threads)))
        return (np.concatenate([p[0] for p in parts]) if parts else np.empty(0, np.int32),
                np.concatenate([p[1] for p in parts]) if parts else np.empty(0, np.int32))


def join(r_key, r_rid, s_key, s_rid) -> tuple[np.ndarray, np.ndarray]:
    """J(R, S): every (rid_R, rid_S) with equal keys, R the build side."""
    with Table(r_key, r_rid) as t:
        return t.probe(s_key, s_rid)


def join_count(r_key, r_rid, s_key) -> int:
    with Table(r_key, r_rid) as t:
        return t.probe_count(s_key)


def oracle_hash(key: int) -> int:
    return int(_load().oracle_hash(int(key)))


def canonical(rid_r, rid_s) -> np.ndarray:
    """The pair multiset as an (M, 2) int32 array sorted by (rid_S, rid_R)."""
    rid_r = np.asarray(rid_r, dtype=np.int32)
    rid_s = np.asarray(rid_s, dtype=np.int32)
    if rid_r.shape != rid_s.shape:
        raise ValueError("pair columns differ in length")
    order = np.lexsort((rid_r, rid_s))
    return np.stack([rid_r[order], rid_s[order]], axis=1)


def match_of(rid_r, rid_s, n_s: int, s_rid=None) -> np.ndarray:
    """Dense form for R with unique keys: ``m[row of s] = rid_R`` or -1.

    ``s_rid`` maps S rows to rids; when omitted, rid_S is the row index.
    Raises if an S row has two matches (R keys not unique)."""
    rid_r = np.asarray(rid_r, dtype=np.int64)
    rid_s = np.asarray(rid_s, dtype=np.int64)
    if s_rid is None:
        row = rid_s
    else:
        inv = np.full(int(np.max(s_rid)) + 1 if len(s_rid) else 0, -1, dtype=np.int64)
        inv[np.asarray(s_rid, dtype=np.int64)] = np.arange(len(s_rid))
        row = inv[rid_s]
    if len(row) and (row.min() < 0 or row.max() >= n_s):
        raise ValueError("rid_S outside S")
    m = np.full(n_s, -1, dtype=np.int64)
    hits = np.bincount(row, minlength=n_s) if len(row) else np.zeros(n_s, dtype=np.int64)
    if len(hits) and hits.max() > 1:
        raise ValueError("an S tuple matched more than once")
    m[row] = rid_r
    return m
