"""Generators: determinism, ranges, bijectivity and distribution shape (CPU)."""
import math

import numpy as np
import pytest

from paper_1307_1955_amd import gen


def test_splitmix64_known_first_output():
    # SplitMix64 started at state 0: the first output is a widely published value.
    assert int(gen.mix64(np.array([gen.GAMMA], dtype=np.uint64))[0]) == 0xE220A8397B1DCDAF
    assert gen.mix64_int(gen.GAMMA) == 0xE220A8397B1DCDAF


@pytest.mark.parametrize("n", [1, 2, 3, 5, 64, 1000, 65539, 1 << 18])
def test_permutation_is_bijection(n):
    p = gen.permutation(7, 1, n)
    assert p.shape == (n,)
    assert np.array_equal(np.sort(p), np.arange(n))


def test_permutation_pointwise_equals_full():
    n = 100003
    full = gen.permutation(11, 3, n)
    part = gen.permutation(11, 3, n, start=5000, count=777)
    assert np.array_equal(full[5000:5777], part)


def test_permutation_depends_on_seed_and_stream():
    a = gen.permutation(1, 1, 4096)
    assert not np.array_equal(a, gen.permutation(2, 1, 4096))
    assert not np.array_equal(a, gen.permutation(1, 2, 4096))
    assert np.array_equal(a, gen.permutation(1, 1, 4096))
    # not the identity, and not a near-identity shift
    assert np.mean(a == np.arange(4096)) < 0.01


def test_uniform_range_and_mean():
    v = gen.uniform_int(5, 2, 0, 1 << 20, 1, 1000)
    assert v.min() == 1 and v.max() == 1000
    assert abs(v.mean() - 500.5) < 5 * 288.7 / math.sqrt(len(v))
    counts = np.bincount(v, minlength=1001)[1:]
    # chi-square against uniform: 999 dof, mean 999, sd ~44.7
    e = len(v) / 1000
    chi2 = ((counts - e) ** 2 / e).sum()
    assert chi2 < 999 + 6 * 44.7


def test_zipf_rank_one_share():
    n, theta, cnt = 1000, 1.0, 1 << 20
    cdf = gen.zipf_cdf(n, theta)
    r = gen.zipf_ranks(9, 4, 0, cnt, cdf)
    assert r.min() >= 1 and r.max() <= n
    h = sum(k ** -theta for k in range(1, n + 1))
    p1 = 1.0 / h
    share = np.mean(r == 1)
    assert abs(share - p1) < 6 * math.sqrt(p1 * (1 - p1) / cnt)
    p2 = 0.5 / h
    assert abs(np.mean(r == 2) - p2) < 6 * math.sqrt(p2 * (1 - p2) / cnt)


def test_zipf_theta_half_rank_one_share():
    n, theta, cnt = 1 << 16, 0.5, 1 << 20
    cdf = gen.zipf_cdf(n, theta)
    r = gen.zipf_ranks(9, 4, 0, cnt, cdf)
    h = float(np.sum(np.arange(1, n + 1, dtype=np.float64) ** -theta))
    p1 = 1.0 / h
    assert abs(np.mean(r == 1) - p1) < 6 * math.sqrt(p1 * (1 - p1) / cnt)


def test_configs_shapes_small():
    r, s = gen.config_c1(n=4096)
    assert len(r) == len(s) == 4096
    assert np.array_equal(np.sort(r.key), np.arange(1, 4097))
    assert np.array_equal(r.rid, np.arange(4096))
    assert s.key.min() >= 1 and s.key.max() <= 4096
    r, s = gen.config_c2(n=1 << 12)
    assert s.key.max() <= 1 << 13
    frac = np.mean(s.key <= 1 << 12)
    assert 0.4 < frac < 0.6


def test_batch_specs_ranges():
    specs = gen.batch_specs(4, 4096)
    nr = np.array([j.n_r for j in specs])
    ns = np.array([j.n_s for j in specs])
    assert nr.min() >= 1024 and nr.max() <= 4194304
    f = ns // nr
    assert np.all(ns == f * nr) and f.min() >= 1 and f.max() <= 16
    # log-uniform: median near the geometric mean 1024 * 64
    med = np.median(nr)
    assert 40000 < med < 100000
    rate = np.array([j.n_r / j.s_domain for j in specs])
    assert rate.min() >= 0.25 - 1e-3 and rate.max() <= 1.0
    assert specs[5].n_r == gen.batch_specs(4, 4096)[5].n_r


def test_job_relations():
    spec = gen.batch_specs(4, 8, r_max=8192)[3]
    r, s = gen.job_relations(spec)
    assert np.array_equal(np.sort(r.key), np.arange(1, spec.n_r + 1))
    assert len(s) == spec.n_s and s.key.max() <= spec.s_domain


def test_poisson_arrivals():
    t = gen.poisson_arrivals(1, 100000, 50.0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps >= 0)
    assert abs(gaps.mean() - 1 / 50.0) < 6 * (1 / 50.0) / math.sqrt(len(gaps))


def test_key_domain_fits_int32():
    gen.check_key_domain((1 << 31) - 1)
    for bad in (0, 1 << 31, 3 << 30):
        with pytest.raises(ValueError):
            gen.uniform_keys(1, 2, 10, bad)


@pytest.mark.parametrize("frac", [0.0, 0.10, 0.25])
def test_skewed_r(frac):
    """Section 5.1's skew sets: exactly round(frac * n) R rows carry the one
    duplicated key, every other key stays unique, S is untouched."""
    n = 10007
    r, s = gen.skewed_r(5, n, 3 * n, 2 * n, frac)
    base_r, base_s = gen.unique_uniform(5, n, 3 * n, 2 * n)
    m = gen.skew_rows(n, frac)
    changed = r.key != base_r.key
    assert np.array_equal(s.key, base_s.key) and np.array_equal(r.rid, base_r.rid)
    # rows set to the key (one of them may have held it already)
    on_key = r.key == gen.SKEW_KEY
    assert on_key.sum() in (m, m + 1) if m else on_key.sum() == 1
    assert changed.sum() in (m, m - 1) if m else changed.sum() == 0
    rest = r.key[~on_key]
    assert len(np.unique(rest)) == len(rest)
    with pytest.raises(ValueError):
        gen.skew_rows(n, 1.5)


@pytest.mark.parametrize("n", [1, 2, 3, 1000, (1 << 20) + 17, 1 << 30])
def test_permutation_index_of_inverts(n):
    rng = np.random.default_rng(n)
    idx = rng.integers(0, n, size=min(n, 5000))
    v = gen.permutation_at(5, 3, n, idx)
    assert np.array_equal(gen.permutation_index_of(5, 3, n, v), idx)
    full = gen.permutation(7, 1, min(n, 4096))
    assert np.array_equal(gen.permutation_index_of(7, 1, min(n, 4096), full), np.arange(min(n, 4096)))
