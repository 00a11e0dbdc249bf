"""Pins for the CPU oracle against things other than itself (CPU only).

* a hand-worked example (tests/golden/worked_example.json);
* a nested-loop brute force on tiny random inputs (duplicates on both sides,
  int32 extremes, empty relations);
* closed forms of the generated workloads (direct addressing through the
  inverse permutation, no hashing);
* a sort-merge join built from numpy's sort and searchsorted;
* the count identity sum_k cnt_R(k) * cnt_S(k);
* the structure of the paper's table (bucket counts sum to |R|, one key node
  per distinct key).
"""
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from paper_1307_1955_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
I32 = st.integers(min_value=-(2 ** 31), max_value=2 ** 31 - 1)


def brute_force(rk, rr, sk, sr):
    out = []
    for j in range(len(sk)):
        for i in range(len(rk)):
            if rk[i] == sk[j]:
                out.append((int(rr[i]), int(sr[j])))
    return sorted(out, key=lambda p: (p[1], p[0]))


def as_list(canon):
    return [tuple(map(int, p)) for p in canon]


def test_worked_example():
    with open(os.path.join(GOLDEN, "worked_example.json")) as f:
        g = json.load(f)
    r_r, r_s = oracle.join(g["R"]["key"], g["R"]["rid"], g["S"]["key"], g["S"]["rid"])
    assert len(r_r) == g["count"]
    assert as_list(oracle.canonical(r_r, r_s)) == sorted(map(tuple, g["pairs"]), key=lambda p: (p[1], p[0]))


@st.composite
def relations(draw):
    pool = draw(st.lists(I32, min_size=1, max_size=12))
    nr = draw(st.integers(0, 60))
    ns = draw(st.integers(0, 60))
    rk = [draw(st.sampled_from(pool)) for _ in range(nr)]
    sk = [draw(st.sampled_from(pool + [0, -1, 2 ** 31 - 1, -(2 ** 31)])) for _ in range(ns)]
    rr = draw(st.lists(I32, min_size=nr, max_size=nr))
    sr = draw(st.lists(I32, min_size=ns, max_size=ns))
    return rk, rr, sk, sr


@settings(max_examples=300, deadline=None)
@given(relations())
def test_oracle_matches_brute_force(rel):
    rk, rr, sk, sr = rel
    o_r, o_s = oracle.join(rk, rr, sk, sr)
    assert as_list(oracle.canonical(o_r, o_s)) == brute_force(rk, rr, sk, sr)
    assert oracle.join_count(rk, rr, sk) == len(o_r)


def test_empty_relations():
    e = np.zeros(0, dtype=np.int32)
    one = np.array([3], dtype=np.int32)
    for rk, sk in [(e, e), (e, one), (one, e)]:
        o_r, o_s = oracle.join(rk, rk, sk, sk)
        assert len(o_r) == 0 and len(o_s) == 0


def test_cartesian_all_equal_keys():
    nr, ns = 37, 53
    rk = np.full(nr, -7, dtype=np.int32)
    sk = np.full(ns, -7, dtype=np.int32)
    rr = np.arange(nr, dtype=np.int32) * 3
    sr = np.arange(ns, dtype=np.int32) + 1000
    o_r, o_s = oracle.join(rk, rr, sk, sr)
    assert len(o_r) == nr * ns
    expect = np.array([(a, b) for b in sr for a in rr], dtype=np.int32)
    assert np.array_equal(oracle.canonical(o_r, o_s), oracle.canonical(expect[:, 0], expect[:, 1]))


def test_probe_emits_in_probe_order_and_build_order():
    # p4 walks S in input order and each key's rid list in R's input order.
    rk = np.array([4, 9, 4, 4], dtype=np.int32)
    rr = np.array([10, 11, 12, 13], dtype=np.int32)
    sk = np.array([9, 4, 8], dtype=np.int32)
    sr = np.array([20, 21, 22], dtype=np.int32)
    o_r, o_s = oracle.join(rk, rr, sk, sr)
    assert o_r.tolist() == [11, 10, 12, 13]
    assert o_s.tolist() == [20, 21, 21, 21]


def test_table_structure():
    rng = np.random.default_rng(0)
    rk = rng.integers(-50, 50, size=1000).astype(np.int32)
    with oracle.Table(rk, np.arange(1000)) as t:
        assert t.nbuckets == 1024
        assert t.nkeys == len(np.unique(rk))
        assert sum(t.bucket_count(b) for b in range(t.nbuckets)) == 1000
        for key in (-50, 0, 49):
            b = oracle.oracle_hash(key) & (t.nbuckets - 1)
            assert t.bucket_count(b) >= np.sum(rk == key)


def closed_form_unique(r_key, s_key):
    """Direct addressing for R keys that are a permutation of 1..|R|: the R row
    holding key k is inv[k]; S rows with keys above |R| have no match."""
    n = len(r_key)
    inv = np.empty(n + 1, dtype=np.int64)
    inv[r_key.astype(np.int64)] = np.arange(n)
    m = np.full(len(s_key), -1, dtype=np.int64)
    hit = s_key.astype(np.int64) <= n
    m[hit] = inv[s_key[hit].astype(np.int64)]
    return m


def test_closed_form_c1_full():
    r, s = gen.config_c1()
    o_r, o_s = oracle.join(r.key, r.rid, s.key, s.rid)
    assert len(o_r) == 1 << 20
    m = oracle.match_of(o_r, o_s, len(s))
    assert np.array_equal(m, closed_form_unique(r.key, s.key))


def test_closed_form_c2_reduced():
    r, s = gen.config_c2(n=1 << 20)
    with oracle.Table(r.key, r.rid) as t:
        cnt = t.probe_count(s.key)
        o_r, o_s = t.probe(s.key, s.rid)
    assert cnt == int(np.sum(s.key <= (1 << 20)))
    m = oracle.match_of(o_r, o_s, len(s))
    assert np.array_equal(m, closed_form_unique(r.key, s.key))


@pytest.mark.slow
def test_closed_form_c2_full_count():
    r, s = gen.config_c2()
    cnt = oracle.join_count(r.key, r.rid, s.key)
    assert cnt == int(np.sum(s.key <= (1 << 24)))
    # binomial(2^24, 1/2): within 6 sd of the mean
    assert abs(cnt - (1 << 23)) < 6 * 2048


def test_zipf_probe_reduced_every_tuple_matches():
    r, s = gen.config_c3(theta=1.0, n_r=1 << 16, n_s=1 << 18)
    o_r, o_s = oracle.join(r.key, r.rid, s.key, s.rid)
    assert len(o_r) == len(s)
    m = oracle.match_of(o_r, o_s, len(s))
    assert np.array_equal(m, closed_form_unique(r.key, s.key))
    # per-key match histogram equals the S key histogram
    keys_matched = r.key[m]
    assert np.array_equal(np.bincount(keys_matched, minlength=(1 << 16) + 1),
                          np.bincount(s.key, minlength=(1 << 16) + 1))


def sort_merge(rk, rr, sk, sr):
    """Many-to-many sort-merge join from numpy primitives."""
    o = np.argsort(rk, kind="stable")
    rk_s, rr_s = rk[o], rr[o]
    lo = np.searchsorted(rk_s, sk, side="left")
    hi = np.searchsorted(rk_s, sk, side="right")
    cnt = hi - lo
    rep_s = np.repeat(np.arange(len(sk)), cnt)
    starts = np.repeat(lo, cnt)
    within = np.arange(len(rep_s)) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    return rr_s[starts + within], sr[rep_s]


def test_sort_merge_with_duplicates():
    rng = np.random.default_rng(12)
    n = 1 << 20
    rk = rng.integers(0, n // 8, size=n // 4).astype(np.int32)  # ~2 duplicates per key
    sk = rng.integers(-1000, n // 6, size=n).astype(np.int32)
    rr = rng.permutation(n // 4).astype(np.int32)
    sr = np.arange(n, dtype=np.int32)
    o_r, o_s = oracle.join(rk, rr, sk, sr)
    m_r, m_s = sort_merge(rk, rr, sk, sr)
    assert len(o_r) == len(m_r)
    assert np.array_equal(oracle.canonical(o_r, o_s), oracle.canonical(m_r, m_s))


def test_count_identity():
    rng = np.random.default_rng(5)
    rk = rng.integers(0, 3000, size=20000).astype(np.int32)
    sk = rng.integers(0, 5000, size=30000).astype(np.int32)
    kr, cr = np.unique(rk, return_counts=True)
    ks, cs = np.unique(sk, return_counts=True)
    common, ir, is_ = np.intersect1d(kr, ks, return_indices=True)
    expect = int(np.sum(cr[ir].astype(np.int64) * cs[is_]))
    assert oracle.join_count(rk, np.arange(len(rk)), sk) == expect


def test_build_side_is_r_even_when_larger():
    rk = np.array([1, 1, 1, 2, 2], dtype=np.int32)
    sk = np.array([1], dtype=np.int32)
    o_r, o_s = oracle.join(rk, np.arange(5), sk, np.array([99]))
    assert sorted(o_r.tolist()) == [0, 1, 2] and o_s.tolist() == [99, 99, 99]


def test_threaded_probe_equals_probe():
    """The probe split over S chunks on several threads (the all-cores CPU
    baseline) returns exactly the single-threaded probe's pairs, in order."""
    rng = np.random.default_rng(77)
    rk = rng.integers(-500, 500, size=3000).astype(np.int32)
    sk = rng.integers(-600, 600, size=7001).astype(np.int32)
    rr = np.arange(3000, dtype=np.int32)
    sr = np.arange(7001, dtype=np.int32) * 5
    with oracle.Table(rk, rr) as t:
        a_r, a_s = t.probe(sk, sr)
        for threads in (1, 3, 8):
            b_r, b_s = t.probe_threads(sk, sr, threads)
            assert np.array_equal(a_r, b_r) and np.array_equal(a_s, b_s)
        e_r, e_s = t.probe_threads(sk[:0], sr[:0], 4)
        assert len(e_r) == 0 and len(e_s) == 0
