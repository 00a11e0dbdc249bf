"""Seeded synthetic relations for the join workloads (host side, numpy).

This module holds only input generation: no hashing, partitioning or joining.
Both the CPU oracle's tests and the GPU path draw their inputs from here, and
``gen.hip`` implements the very same counter-based definitions on the device
so that large relations can be produced in HBM and still be regenerated on
the host, row for row, for checking.

Every value is a pure function of ``(seed, stream, index)``:

* ``mix64`` is the output function of SplitMix64 (Steele, Lea & Flood,
  "Fast splittable pseudorandom number generators", OOPSLA 2014); the i-th
  draw of a stream is ``mix64(key + (i + 1) * GAMMA)``, i.e. the i-th output of
  a SplitMix64 generator whose state starts at ``key``.
* A random permutation of ``[0, n)`` is a 4-round Feistel network on the
  smallest even-bit domain covering ``n`` plus cycle walking (Luby & Rackoff
  1988; Black & Rogaway 2002), so any single element can be computed alone.
* Zipf ranks are drawn by inversion of a float64 CDF table (binary search for
  the first entry above the uniform variate).

Workload shapes follow the paper's evaluation setup (Section 5.1): two 4-byte
integer attributes per tuple, a 16M-tuple default relation, uniform keys, and
selectivity varied around 50%.  The paper's own data generator is not
available; these relations stand in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_STREAM_MUL = 0xD1B54A32D192ED03

# Stream identifiers; a job j of a batch uses (j + 1) << 8 | kind.
STREAM_R_KEYS = 1
STREAM_S_KEYS = 2
STREAM_JOB_SIZE = 3
STREAM_JOB_FACTOR = 4
STREAM_JOB_MATCH = 5
STREAM_ARRIVALS = 6
STREAM_SKEW_ROWS = 7


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def mix64_int(x: int) -> int:
    """Scalar version of :func:`mix64` on a Python int."""
    z = x & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int) -> int:
    """Starting state of stream ``stream`` under ``seed``."""
    return mix64_int(mix64_int((seed + GAMMA) & MASK64) ^ ((stream * _STREAM_MUL) & MASK64))


def draws_at(seed: int, stream: int, idx) -> np.ndarray:
    """Draws number ``idx`` (any uint64 index array) of a stream."""
    key = stream_key(seed, stream)
    i = np.asarray(idx, dtype=np.uint64) + np.uint64(1)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + i * np.uint64(GAMMA)
    return mix64(z)


def draws(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """Draws ``start .. start+count-1`` of a stream as uint64."""
    return draws_at(seed, stream, np.arange(start, start + count, dtype=np.uint64))


def _uniform_from(d: np.ndarray, lo: int, m: int) -> np.ndarray:
    if not (1 <= m <= (1 << 32)):
        raise ValueError("range size must be in [1, 2^32]")
    d = d >> np.uint64(32)
    with np.errstate(over="ignore"):
        v = (d * np.uint64(m)) >> np.uint64(32)
    return v.astype(np.int64) + lo


def uniform_int(seed: int, stream: int, start: int, count: int, lo: int, m: int) -> np.ndarray:
    """Integers in ``[lo, lo + m)`` by multiply-shift of the draw's top 32 bits."""
    return _uniform_from(draws(seed, stream, start, count), lo, m)


def uniform_int_at(seed: int, stream: int, idx, lo: int, m: int) -> np.ndarray:
    return _uniform_from(draws_at(seed, stream, idx), lo, m)


def _unit_from(d: np.ndarray) -> np.ndarray:
    return (d >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def unit_float(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """Floats in ``[0, 1)`` with 53 random bits."""
    return _unit_from(draws(seed, stream, start, count))


def _feistel_half_bits(n: int) -> int:
    bits = max(1, (n - 1).bit_length())
    return max(1, (bits + 1) // 2)


def feistel_round_keys(seed: int, stream: int) -> list[int]:
    key = stream_key(seed, stream)
    return [mix64_int((key + (r + 1) * GAMMA) & MASK64) for r in range(4)]


def feistel_half_bits(n: int) -> int:
    """Half width h of the Feistel domain 2^(2h) used for a permutation of [0, n)."""
    return _feistel_half_bits(n)


def permutation_at(seed: int, stream: int, n: int, idx) -> np.ndarray:
    """Elements ``idx`` (index array into [0, n)) of a pseudo-random permutation of ``[0, n)``."""
    x = np.asarray(idx, dtype=np.uint64)
    if n <= 0 or x.size == 0:
        return np.zeros(0, dtype=np.int64)
    h = _feistel_half_bits(n)
    mask = np.uint64((1 << h) - 1)
    rk = [np.uint64(k) for k in feistel_round_keys(seed, stream)]

    def enc(v: np.ndarray) -> np.ndarray:
        left = v >> np.uint64(h)
        right = v & mask
        for r in range(4):
            f = mix64(rk[r] ^ right) & mask
            left, right = right, left ^ f
        return (left << np.uint64(h)) | right

    y = enc(x)
    bad = y >= np.uint64(n)
    while bad.any():
        y[bad] = enc(y[bad])
        bad = y >= np.uint64(n)
    return y.astype(np.int64)


def permutation_index_of(seed: int, stream: int, n: int, values) -> np.ndarray:
    """Inverse of ``permutation_at``: the index at which the permutation of
    ``[0, n)`` holds each of ``values`` (the Feistel rounds run backwards, with
    the same cycle walking until the result lies in ``[0, n)``)."""
    y = np.asarray(values, dtype=np.uint64)
    if n <= 0 or y.size == 0:
        return np.zeros(0, dtype=np.int64)
    h = _feistel_half_bits(n)
    mask = np.uint64((1 << h) - 1)
    rk = [np.uint64(k) for k in feistel_round_keys(seed, stream)]

    def dec(v: np.ndarray) -> np.ndarray:
        left = v >> np.uint64(h)
        right = v & mask
        for r in range(3, -1, -1):
            f = mix64(rk[r] ^ left) & mask
            left, right = right ^ f, left
        return (left << np.uint64(h)) | right

    x = dec(y)
    bad = x >= np.uint64(n)
    while bad.any():
        x[bad] = dec(x[bad])
        bad = x >= np.uint64(n)
    return x.astype(np.int64)


def permutation(seed: int, stream: int, n: int, start: int = 0, count: int | None = None) -> np.ndarray:
    """Elements ``start .. start+count-1`` of a pseudo-random permutation of ``[0, n)``."""
    if count is None:
        count = n - start
    if n <= 0 or count <= 0:
        return np.zeros(0, dtype=np.int64)
    return permutation_at(seed, stream, n, np.arange(start, start + count, dtype=np.uint64))


def zipf_cdf(n: int, theta: float) -> np.ndarray:
    """CDF table of Zipf(theta) over ranks 1..n; the last entry is exactly 1."""
    k = np.arange(1, n + 1, dtype=np.float64)
    w = k ** (-float(theta))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    cdf[-1] = 1.0
    return cdf


def _zipf_from(d: np.ndarray, cdf: np.ndarray) -> np.ndarray:
    u = _unit_from(d)
    idx = np.searchsorted(cdf, u, side="right")
    np.minimum(idx, len(cdf) - 1, out=idx)
    return idx.astype(np.int64) + 1


def zipf_ranks(seed: int, stream: int, start: int, count: int, cdf: np.ndarray) -> np.ndarray:
    """Zipf ranks (1-based): the first index whose CDF entry exceeds the variate, plus one."""
    return _zipf_from(draws(seed, stream, start, count), cdf)


def zipf_ranks_at(seed: int, stream: int, idx, cdf: np.ndarray) -> np.ndarray:
    return _zipf_from(draws_at(seed, stream, idx), cdf)


# ---------------------------------------------------------------------------
# Relations
# ---------------------------------------------------------------------------


@dataclass
class Relation:
    """SoA relation: int32 ``key`` and ``rid`` arrays of equal length."""

    key: np.ndarray
    rid: np.ndarray

    def __post_init__(self):
        self.key = np.ascontiguousarray(self.key, dtype=np.int32)
        self.rid = np.ascontiguousarray(self.rid, dtype=np.int32)
        if self.key.shape != self.rid.shape or self.key.ndim != 1:
            raise ValueError("key and rid must be 1-D arrays of equal length")

    def __len__(self) -> int:
        return int(self.key.shape[0])


def rows(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.int32)


def perm_keys(seed: int, stream: int, n: int) -> np.ndarray:
    """Unique keys: a seeded permutation of ``1..n``."""
    return (permutation(seed, stream, n) + 1).astype(np.int32)


INT32_MAX = (1 << 31) - 1


def check_key_domain(domain: int) -> None:
    """Keys 1..domain must be int32 values."""
    if not 1 <= domain <= INT32_MAX:
        raise ValueError("key domain 1..%d does not fit int32 keys" % domain)


def uniform_keys(seed: int, stream: int, count: int, domain: int) -> np.ndarray:
    """Keys drawn uniformly from ``1..domain`` (domain <= 2^31 - 1)."""
    check_key_domain(domain)
    return uniform_int(seed, stream, 0, count, 1, domain).astype(np.int32)


def unique_uniform(seed: int, n_r: int, n_s: int, s_domain: int) -> tuple[Relation, Relation]:
    """R keys a permutation of 1..n_r, rid = row; S keys uniform over 1..s_domain."""
    r = Relation(perm_keys(seed, STREAM_R_KEYS, n_r), rows(n_r))
    s = Relation(uniform_keys(seed, STREAM_S_KEYS, n_s, s_domain), rows(n_s))
    return r, s


SKEW_KEY = 1


def skew_rows(n_r: int, frac: float) -> int:
    """Rows of an n_r-tuple R that carry the one duplicated key at fraction frac."""
    if not 0.0 <= frac <= 1.0:
        raise ValueError("skew fraction must lie in [0, 1]")
    return int(round(frac * n_r))


def skewed_r(seed: int, n_r: int, n_s: int, s_domain: int, frac: float) -> tuple[Relation, Relation]:
    """The skewed sets of Section 5.1: ``unique_uniform`` with a fraction ``frac``
    of R's rows (the rows whose index under a seeded permutation is below
    ``round(frac * n_r)``) set to the one key ``SKEW_KEY``; every other R key
    stays unique.  Low skew is frac = 0.10, high skew 0.25."""
    r, s = unique_uniform(seed, n_r, n_s, s_domain)
    m = skew_rows(n_r, frac)
    if m:
        r.key[permutation(seed, STREAM_SKEW_ROWS, n_r) < m] = SKEW_KEY
    return r, s


def config_c1(seed: int = 1, n: int = 1 << 20) -> tuple[Relation, Relation]:
    """SHJ check workload: |R| = |S| = n, every S key drawn from R's keys."""
    return unique_uniform(seed, n, n, n)


def config_c2(seed: int = 2, n: int = 1 << 24) -> tuple[Relation, Relation]:
    """16M x 16M: R keys unique over 1..n, S keys uniform over 1..2n (about 50% match)."""
    return unique_uniform(seed, n, n, 2 * n)


def config_c3(seed: int = 3, theta: float = 1.0, n_r: int = 1 << 24, n_s: int = 1 << 26) -> tuple[Relation, Relation]:
    """Skewed probe: S keys Zipf(theta) over R's keys (rank k is key k)."""
    r = Relation(perm_keys(seed, STREAM_R_KEYS, n_r), rows(n_r))
    cdf = zipf_cdf(n_r, theta)
    s = Relation(zipf_ranks(seed, STREAM_S_KEYS, 0, n_s, cdf).astype(np.int32), rows(n_s))
    return r, s


# ---------------------------------------------------------------------------
# Batches of independent joins
# ---------------------------------------------------------------------------

JOB_R_MIN = 1024
JOB_R_MAX = 4194304


@dataclass
class JobSpec:
    """Sizes of one join of a batch: |R|, |S| = factor * |R|, S keys over 1..s_domain."""

    index: int
    n_r: int
    n_s: int
    s_domain: int
    seed: int

    @property
    def r_stream(self) -> int:
        return ((self.index + 1) << 8) | STREAM_R_KEYS

    @property
    def s_stream(self) -> int:
        return ((self.index + 1) << 8) | STREAM_S_KEYS


def batch_specs(seed: int, njobs: int, r_min: int = JOB_R_MIN, r_max: int = JOB_R_MAX,
                max_factor: int = 16) -> list[JobSpec]:
    """Job sizes: |R| log-uniform in [r_min, r_max], |S| = |R| * U{1..max_factor},
    S keys uniform over 1..ceil(|R| / m) with m ~ U[0.25, 1] (a 25-100% match rate)."""
    u = unit_float(seed, STREAM_JOB_SIZE, 0, njobs)
    ratio = r_max / r_min
    n_r = np.clip(np.round(r_min * np.power(ratio, u)), r_min, r_max).astype(np.int64)
    factor = uniform_int(seed, STREAM_JOB_FACTOR, 0, njobs, 1, max_factor)
    m = 0.25 + 0.75 * unit_float(seed, STREAM_JOB_MATCH, 0, njobs)
    specs = []
    for j in range(njobs):
        nr = int(n_r[j])
        dom = int(math.ceil(nr / float(m[j])))
        specs.append(JobSpec(j, nr, nr * int(factor[j]), max(dom, nr), seed))
    return specs


def job_relations(spec: JobSpec) -> tuple[Relation, Relation]:
    """Host copy of one batch job's relations (same values the device generator writes)."""
    r = Relation(perm_keys(spec.seed, spec.r_stream, spec.n_r), rows(spec.n_r))
    s = Relation(uniform_keys(spec.seed, spec.s_stream, spec.n_s, spec.s_domain), rows(spec.n_s))
    return r, s


def poisson_arrivals(seed: int, count: int, qps: float) -> np.ndarray:
    """Arrival times (seconds from 0) of an open-loop Poisson process at rate ``qps``."""
    u = unit_float(seed, STREAM_ARRIVALS, 0, count)
    gaps = -np.log1p(-u) / float(qps)
    return np.cumsum(gaps)
