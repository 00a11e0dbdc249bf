"""GPU tests of the join of host-resident relations larger than the device can
hold (hj_join_external): partition pass in chunks, linked partition pairs,
pairs joined on the device.  Small workspaces force many chunks, a fan-out and
S pieces; results against the oracle in full.  One relation pair larger than
the device's free memory (a ballast allocation leaves less free than the pair
needs) is checked completely by its closed form and against the oracle on
sampled S rows."""
import numpy as np
import pytest

import oracle
from paper_1307_1955_amd import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1307_1955_amd.hj as hj  # noqa: E402
from paper_1307_1955_amd.gen import device as dgen  # noqa: E402

DEV = torch.device("cuda:0")


def external(p, rk, rr, sk, sr, ws_bytes, cap):
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=DEV)
    o_r = np.full(max(cap, 1), -5, dtype=np.int32)
    o_s = np.full(max(cap, 1), -5, dtype=np.int32)
    cnt, info = hj.hj_join_external(p, rk, rr, sk, sr, o_r[:cap], o_s[:cap], ws)
    return o_r[:cnt], o_s[:cnt], cnt, info


def dup_relations(seed, n_r, n_s, domain):
    rng = np.random.default_rng(seed)
    rk = rng.integers(-domain // 2, domain // 2, size=n_r).astype(np.int64)
    sk = rng.integers(-domain // 2, domain // 2 + domain // 4, size=n_s).astype(np.int64)
    ext = np.array([-(2 ** 31), 2 ** 31 - 1, 0, -1], dtype=np.int64)
    rk[: len(ext)] = ext
    sk[-len(ext):] = ext[::-1]
    rr = (rng.permutation(n_r).astype(np.int32) * 3 + 1).astype(np.int32)
    sr = (rng.permutation(n_s).astype(np.int32) - 5).astype(np.int32)
    return rk.astype(np.int32), rr, sk.astype(np.int32), sr


@pytest.mark.parametrize("kw", [dict(algo="auto", one_pass=True), dict(algo="phj", passes=2, bits=(5, 5)),
                                dict(algo="shj")], ids=["auto", "phj2_5_5", "shj"])
def test_external_small_workspace_vs_oracle(kw):
    """4M x 6M with duplicates through a 64 MiB workspace: a fan-out and many chunks."""
    p = hj.params(**kw)
    rk, rr, sk, sr = dup_relations(91, 4_000_037, 6_000_011, 3_000_000)
    want_r, want_s = oracle.join(rk, rr, sk, sr)
    got_r, got_s, cnt, info = external(p, rk, rr, sk, sr, 64 << 20, len(want_r) + 10)
    assert info["fanout_bits"] >= 1 and info["pieces"] >= 2, info
    assert cnt == len(want_r)
    assert np.array_equal(oracle.canonical(got_r, got_s), oracle.canonical(want_r, want_s))


def test_external_fits_in_one_piece():
    """A workspace large enough for the whole join: no partition pass (fan-out 0)."""
    p = hj.params("auto", one_pass=True)
    r, s = gen.unique_uniform(92, 1 << 20, 3 << 20, 1 << 21)
    want_r, want_s = oracle.join(r.key, r.rid, s.key, s.rid)
    got_r, got_s, cnt, info = external(p, r.key, r.rid, s.key, s.rid, 1 << 30, len(s))
    assert info["fanout_bits"] == 0 and info["pieces"] == 1 and info["partition_s"] == 0.0
    assert np.array_equal(oracle.canonical(got_r, got_s), oracle.canonical(want_r, want_s))


def test_external_skewed_s_in_pieces():
    """Zipf(1.0) S over a 1M R: the partition holding the most frequent keys is far
    larger than the rest and is joined in S pieces."""
    p = hj.params("auto", one_pass=True)
    n_r, n_s = 1 << 20, 12 << 20
    r = gen.Relation(gen.perm_keys(93, gen.STREAM_R_KEYS, n_r).astype(np.int32), gen.rows(n_r))
    cdf = gen.zipf_cdf(n_r, 1.0)
    sk = gen.zipf_ranks(93, gen.STREAM_S_KEYS, 0, n_s, cdf).astype(np.int32)
    sr = gen.rows(n_s)
    want = oracle.match_of(*oracle.join(r.key, r.rid, sk, sr), n_s)
    got_r, got_s, cnt, info = external(p, r.key, r.rid, sk, sr, 64 << 20, n_s)
    assert cnt == n_s and info["fanout_bits"] >= 1
    assert np.array_equal(oracle.match_of(got_r, got_s, n_s), want)


def test_external_capacity():
    """Too small an output: the full count is reported (HJ_ERR_CAPACITY), nothing
    is written past capacity, and every pair written is a pair of the join."""
    p = hj.params("auto", one_pass=True)
    r, s = gen.unique_uniform(94, 3 << 20, 5 << 20, 6 << 20)
    want = oracle.join_count(r.key, r.rid, s.key)
    cap = want // 3
    ws = torch.empty(64 << 20, dtype=torch.uint8, device=DEV)
    o_r = np.full(want, -5, dtype=np.int32)
    o_s = np.full(want, -5, dtype=np.int32)
    with pytest.raises(hj.HJError) as e:
        hj.hj_join_external(p, r.key, r.rid, s.key, s.rid, o_r[:cap], o_s[:cap], ws)
    assert e.value.status == hj.HJ_ERR_CAPACITY
    assert str(want) in e.value.message
    assert np.all(o_r[cap:] == -5) and np.all(o_s[cap:] == -5)
    assert np.array_equal(r.key[o_r[:cap]], s.key[o_s[:cap]])  # rid = row index


def test_external_larger_than_free_device_memory():
    """|R| = |S| = 2^30 (16 GB of input) with less than that free on the device: a
    ballast allocation leaves 12 GiB free and the join gets an 8 GiB workspace.
    Checked in full by the closed form (count, every pair joins equal keys, no S
    row twice) and against the oracle on sampled S rows."""
    n = 1 << 30
    seed = 95
    # inputs made on the device, kept in pinned host memory
    hk = {}
    for name, make in (("rk", lambda: dgen.perm_keys(seed, gen.STREAM_R_KEYS, n, DEV)),
                       ("sk", lambda: dgen.uniform_keys(seed, gen.STREAM_S_KEYS, n, 2 * n - 1, DEV))):
        t = make()
        hk[name] = torch.empty(n, dtype=torch.int32, pin_memory=True)
        hk[name].copy_(t)
        del t
    rows = torch.empty(n, dtype=torch.int32, pin_memory=True)
    rows.copy_(dgen.rows(n, DEV))
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    rk, sk = hk["rk"].numpy(), hk["sk"].numpy()
    want = int(np.count_nonzero(sk <= n))
    free, _ = torch.cuda.mem_get_info()
    ballast = torch.empty(max(0, free - (12 << 30)), dtype=torch.uint8, device=DEV)
    free, _ = torch.cuda.mem_get_info()
    assert free < 16 * n  # the pair does not fit the free device memory
    ws = torch.empty(8 << 30, dtype=torch.uint8, device=DEV)
    o_r = torch.empty(want + 1024, dtype=torch.int32, pin_memory=True)
    o_s = torch.empty(want + 1024, dtype=torch.int32, pin_memory=True)
    p = hj.params("auto", one_pass=True)
    cnt, info = hj.hj_join_external(p, hk["rk"], rows, hk["sk"], rows, o_r, o_s, ws)
    del ws, ballast
    torch.cuda.empty_cache()
    print("external 2^30 x 2^30: %s, %.3g tuples/s including host transfers"
          % (info, 2 * n / info["total_s"]), flush=True)
    assert info["fanout_bits"] >= 1
    assert cnt == want
    a, b = o_r[:cnt].numpy(), o_s[:cnt].numpy()
    assert a.min() >= 0 and a.max() < n and b.min() >= 0 and b.max() < n
    for lo in range(0, cnt, 1 << 27):  # every pair joins equal keys (rid = row index)
        hi = min(cnt, lo + (1 << 27))
        assert np.array_equal(rk[a[lo:hi]], sk[b[lo:hi]])
    seen = np.zeros(n, dtype=np.bool_)
    seen[b] = True
    assert int(np.count_nonzero(seen)) == cnt  # no S row twice
    del seen
    # the oracle on sampled S rows: their R partners are the rows whose keys they
    # carry (R keys are a permutation of 1..n, found by inverting it)
    rows_s = np.sort(np.random.default_rng(96).choice(n, size=1 << 16, replace=False))
    keys = sk[rows_s]
    hit = keys <= n
    # (two sampled S rows may carry one key: R' holds each R row once)
    r_rows = np.unique(gen.permutation_index_of(seed, gen.STREAM_R_KEYS, n, keys[hit].astype(np.int64) - 1))
    assert np.array_equal(np.sort(rk[r_rows]), np.unique(keys[hit]))
    w_r, w_s = oracle.join(rk[r_rows], r_rows.astype(np.int32), keys, rows_s.astype(np.int32))
    m = np.full(n, -1, dtype=np.int32)
    m[b] = a
    got = np.stack([m[rows_s], rows_s], axis=1)
    got = got[got[:, 0] >= 0]
    assert np.array_equal(oracle.canonical(got[:, 0], got[:, 1]), oracle.canonical(w_r, w_s))
