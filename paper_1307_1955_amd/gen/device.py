"""Device-side generation (libhjgen.so) of the relations defined in ``gen``.

Produces in HBM exactly the values the numpy functions of ``gen`` compute, so
full-size relations need no host generation or upload; tests regenerate any
sampled rows on the host to check.  Holds no join arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np
import torch

from . import (SKEW_KEY, STREAM_R_KEYS, STREAM_S_KEYS, STREAM_SKEW_ROWS, JobSpec, check_key_domain,
               feistel_half_bits, feistel_round_keys, skew_rows, stream_key, zipf_cdf)

LIB_PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "libhjgen.so")
_lock = threading.Lock()
_lib = None


def load() -> ctypes.CDLL:
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise FileNotFoundError("%s is missing: build it with `python -m paper_1307_1955_amd.build`"
                                        % LIB_PATH)
            lib = ctypes.CDLL(LIB_PATH)
            vp, u64, i64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32
            lib.hjgen_perm_keys.argtypes = [vp, u64, ctypes.POINTER(u64), u32, i64, vp]
            lib.hjgen_uniform.argtypes = [vp, u64, u64, i64, u64, vp]
            lib.hjgen_zipf.argtypes = [vp, u64, u64, vp, u64, vp]
            lib.hjgen_iota.argtypes = [vp, u64, i64, vp]
            for f in (lib.hjgen_perm_keys, lib.hjgen_uniform, lib.hjgen_zipf, lib.hjgen_iota):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def _s() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ok(rc: int) -> None:
    if rc != 0:
        raise RuntimeError("device generator failed (code %d)" % rc)


def perm_keys(seed: int, stream: int, n: int, device="cuda", out: torch.Tensor | None = None) -> torch.Tensor:
    """1 + a seeded permutation of [0, n) (unique keys 1..n), as int32 on the device."""
    out = torch.empty(n, dtype=torch.int32, device=device) if out is None else out
    if n:
        rk = (ctypes.c_uint64 * 4)(*feistel_round_keys(seed, stream))
        _ok(load().hjgen_perm_keys(out.data_ptr(), n, rk, feistel_half_bits(n), 1, _s()))
    return out


def uniform_keys(seed: int, stream: int, count: int, domain: int, device="cuda",
                 out: torch.Tensor | None = None) -> torch.Tensor:
    check_key_domain(domain)
    out = torch.empty(count, dtype=torch.int32, device=device) if out is None else out
    if count:
        _ok(load().hjgen_uniform(out.data_ptr(), count, stream_key(seed, stream), 1, domain, _s()))
    return out


def zipf_keys(seed: int, stream: int, count: int, cdf: torch.Tensor, device="cuda",
              out: torch.Tensor | None = None) -> torch.Tensor:
    if cdf.dtype != torch.float64 or not cdf.is_cuda:
        raise ValueError("cdf must be a float64 CUDA tensor")
    out = torch.empty(count, dtype=torch.int32, device=device) if out is None else out
    if count:
        _ok(load().hjgen_zipf(out.data_ptr(), count, stream_key(seed, stream), cdf.data_ptr(), cdf.numel(), _s()))
    return out


def rows(n: int, device="cuda", out: torch.Tensor | None = None) -> torch.Tensor:
    out = torch.empty(n, dtype=torch.int32, device=device) if out is None else out
    if n:
        _ok(load().hjgen_iota(out.data_ptr(), n, 0, _s()))
    return out


def unique_uniform(seed: int, n_r: int, n_s: int, s_domain: int, device="cuda"):
    """Device tensors (r_key, r_rid, s_key, s_rid) equal to ``gen.unique_uniform``."""
    return (perm_keys(seed, STREAM_R_KEYS, n_r, device), rows(n_r, device),
            uniform_keys(seed, STREAM_S_KEYS, n_s, s_domain, device), rows(n_s, device))


def skewed_r(seed: int, n_r: int, n_s: int, s_domain: int, frac: float, device="cuda"):
    """Device tensors equal to ``gen.skewed_r``."""
    rk, rr, sk, sr = unique_uniform(seed, n_r, n_s, s_domain, device)
    m = skew_rows(n_r, frac)
    if m:
        sel = perm_keys(seed, STREAM_SKEW_ROWS, n_r, device)  # 1 + the row's permuted index
        rk.masked_fill_(sel <= m, SKEW_KEY)
        del sel
    return rk, rr, sk, sr


def config_c1(seed: int = 1, n: int = 1 << 20, device="cuda"):
    return unique_uniform(seed, n, n, n, device)


def config_c2(seed: int = 2, n: int = 1 << 24, device="cuda"):
    return unique_uniform(seed, n, n, 2 * n, device)


def config_c3(seed: int = 3, theta: float = 1.0, n_r: int = 1 << 24, n_s: int = 1 << 26, device="cuda"):
    cdf = torch.from_numpy(zipf_cdf(n_r, theta)).to(device)
    sk = zipf_keys(seed, STREAM_S_KEYS, n_s, cdf, device)
    del cdf
    return perm_keys(seed, STREAM_R_KEYS, n_r, device), rows(n_r, device), sk, rows(n_s, device)


def job_relations(spec: JobSpec, device="cuda"):
    return (perm_keys(spec.seed, spec.r_stream, spec.n_r, device), rows(spec.n_r, device),
            uniform_keys(spec.seed, spec.s_stream, spec.n_s, spec.s_domain, device), rows(spec.n_s, device))
