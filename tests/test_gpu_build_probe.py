"""GPU parity of the split join: hj_build over R once, then hj_probe with
several relations S (Algorithm 1's build and probe phases as separate calls).
Every probe must give the multiset of pairs the oracle gives for (R, S), and
the same as hj_join with the table's parameters."""
import numpy as np
import pytest

import oracle
from paper_1307_1955_amd import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1307_1955_amd.hj as hj  # noqa: E402

DEV = torch.device("cuda:0")


def to_dev(*arrays):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV) for a in arrays]


def dup_relations(seed, n_r, n_s, domain):
    """Duplicates on both sides, negative keys and the int32 extremes."""
    rng = np.random.default_rng(seed)
    rk = rng.integers(-domain // 2, domain // 2, size=n_r).astype(np.int64)
    sk = rng.integers(-domain // 2, domain // 2 + domain // 4, size=n_s).astype(np.int64)
    ext = np.array([-(2 ** 31), 2 ** 31 - 1, 0, -1], dtype=np.int64)
    rk[: len(ext)] = ext
    sk[-len(ext):] = ext[::-1]
    rr = rng.permutation(n_r).astype(np.int32) * 3 + 1
    sr = rng.permutation(n_s).astype(np.int32) - 5
    return rk.astype(np.int32), rr, sk.astype(np.int32), sr


def canon(o_r, o_s):
    return oracle.canonical(o_r.cpu().numpy(), o_s.cpu().numpy())


CASES = [
    ("shj", dict(algo="shj")),
    ("shj_1pass", dict(algo="shj", one_pass=True)),
    ("phj1_b7", dict(algo="phj", passes=1, bits=(7,))),
    ("phj2_6_5", dict(algo="phj", passes=2, bits=(6, 5))),
    ("phj2_6_6_1pass", dict(algo="phj", passes=2, bits=(6, 6), one_pass=True)),
    ("phj2_5_5_murmur_t1024", dict(algo="phj", passes=2, bits=(5, 5), hash="murmur2", tile=1024)),
    ("phj2_3_3_ldscap256", dict(algo="phj", passes=2, bits=(3, 3), lds_cap=256)),
    ("phj1_4_ldscap256_1pass", dict(algo="phj", passes=1, bits=(4,), lds_cap=256, one_pass=True)),
    ("auto", dict(algo="auto")),
    ("auto_1pass", dict(algo="auto", one_pass=True)),
]


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_build_once_probe_many(name, kw):
    rk, rr, sk1, sr1 = dup_relations(41, 30011, 50021, 20000)
    _, _, sk2, sr2 = dup_relations(42, 10, 77777, 20000)
    p = hj.params(**kw)
    R = to_dev(rk, rr)
    tab = hj.Table(*R, p=p)
    assert tab.params.algo in (hj.HJ_SHJ, hj.HJ_PHJ) and tab.params.tile != 0
    for sk, sr in ((sk1, sr1), (sk2, sr2), (sk1[:999], sr1[:999])):
        S = to_dev(sk, sr)
        o_r, o_s, cnt = tab.probe(*S)
        want_r, want_s = oracle.join(rk, rr, sk, sr)
        assert cnt == len(want_r), (cnt, len(want_r))
        got = canon(o_r, o_s)
        assert np.array_equal(got, oracle.canonical(want_r, want_s))
        # hj_join with the table's (resolved) parameters gives the same multiset
        j_r, j_s, j_c = hj.join(*R, *S, p=tab.params)
        assert j_c == cnt and np.array_equal(canon(j_r, j_s), got)


def test_direct_table_reads_r():
    """PHJ with passes 0: the table is R itself."""
    r, s = gen.unique_uniform(43, 3000, 20000, 4000)
    R = to_dev(r.key, r.rid)
    tab = hj.Table(*R, p=hj.params("phj", 0, (0, 0)))
    assert tab.params.passes == 0 and tab.params.lds_cap >= 3000
    o_r, o_s, cnt = tab.probe(*to_dev(s.key, s.rid))
    want_r, want_s = oracle.join(r.key, r.rid, s.key, s.rid)
    assert cnt == len(want_r)
    assert np.array_equal(canon(o_r, o_s), oracle.canonical(want_r, want_s))


@pytest.mark.parametrize("kw", [dict(algo="phj", passes=2, bits=(6, 6)), dict(algo="phj", passes=1, bits=(6,))])
def test_partitioned_table_holds_r(kw):
    """PHJ with 1 or 2 passes keeps R's partitions in the table: overwriting R's
    arrays after the build changes no probe result."""
    r, s = gen.unique_uniform(44, 50000, 80000, 60000)
    rk, rr = to_dev(r.key, r.rid)
    tab = hj.Table(rk, rr, p=hj.params(**kw))
    torch.cuda.synchronize()
    rk.fill_(7)
    rr.fill_(-1)
    o_r, o_s, cnt = tab.probe(*to_dev(s.key, s.rid))
    want_r, want_s = oracle.join(r.key, r.rid, s.key, s.rid)
    assert cnt == len(want_r)
    assert np.array_equal(canon(o_r, o_s), oracle.canonical(want_r, want_s))


def test_probes_on_two_streams():
    """Probes of one table run concurrently on two streams with their own workspaces."""
    r, s1 = gen.unique_uniform(45, 40000, 90000, 80000)
    _, s2 = gen.unique_uniform(46, 10, 70000, 50000)
    R = to_dev(r.key, r.rid)
    tab = hj.Table(*R, p=hj.params("phj", 2, (5, 6), one_pass=True))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ins = [to_dev(s1.key, s1.rid), to_dev(s2.key, s2.rid)]
    outs, counts = [], []
    for st, S in zip(streams, ins):
        ws = tab.probe_workspace(S[0].numel())
        o = (torch.empty(S[0].numel(), dtype=torch.int32, device=DEV),
             torch.empty(S[0].numel(), dtype=torch.int32, device=DEV))
        d = torch.zeros(1, dtype=torch.int64, device=DEV)
        hj.hj_probe(tab.t, *S, *o, ws, d, stream=st)
        outs.append((o, ws))
        counts.append(d)
    torch.cuda.synchronize()
    for (o, _), d, s in zip(outs, counts, (s1, s2)):
        c = int(d.item())
        want_r, want_s = oracle.join(r.key, r.rid, s.key, s.rid)
        assert c == len(want_r)
        assert np.array_equal(canon(o[0][:c], o[1][:c]), oracle.canonical(want_r, want_s))


@pytest.mark.parametrize("kw", [dict(algo="shj"), dict(algo="phj", passes=2, bits=(4, 4)),
                                dict(algo="phj", passes=0, bits=(0, 0))])
def test_empty_sides(kw):
    e = np.zeros(0, dtype=np.int32)
    one = np.array([5], dtype=np.int32)
    for rk, sk in ((e, one), (one, e), (e, e), (one, one)):
        tab = hj.Table(*to_dev(rk, np.arange(len(rk))), p=hj.params(**kw))
        o_r, o_s, cnt = tab.probe(*to_dev(sk, np.arange(len(sk)) + 3))
        assert cnt == (1 if len(rk) and len(sk) else 0)
        if cnt:
            assert (int(o_r[0]), int(o_s[0])) == (0, 3)


@pytest.mark.parametrize("kw", [dict(algo="shj"), dict(algo="phj", passes=2, bits=(6, 6)),
                                dict(algo="phj", passes=2, bits=(6, 6), one_pass=True)])
def test_probe_capacity_guard(kw):
    r, s = gen.unique_uniform(47, 30000, 60000, 40000)
    tab = hj.Table(*to_dev(r.key, r.rid), p=hj.params(**kw))
    S = to_dev(s.key, s.rid)
    want = oracle.join_count(r.key, r.rid, s.key)
    cap = want // 3
    buf_r = torch.full((want,), -7, dtype=torch.int32, device=DEV)
    buf_s = torch.full((want,), -7, dtype=torch.int32, device=DEV)
    ws = tab.probe_workspace(len(s))
    d = torch.zeros(1, dtype=torch.int64, device=DEV)
    hj.hj_probe(tab.t, *S, buf_r[:cap], buf_s[:cap], ws, d)
    torch.cuda.synchronize()
    assert int(d.item()) == want
    assert torch.all(buf_r[cap:] == -7) and torch.all(buf_s[cap:] == -7)


@pytest.mark.parametrize("algo", ["phj", "shj"])
def test_r_side_skew_overflow(algo):
    """A quarter of R shares one key: for PHJ an R partition beyond the LDS budget
    takes the HBM-table path inside the probe; for SHJ the key's chain is long
    enough for the block-wide scan of R."""
    n_r, n_s = 1 << 17, 1 << 18
    r, s = gen.unique_uniform(48, n_r, n_s, 2 * n_r)
    rk = r.key.copy()
    rng = np.random.default_rng(5)
    rk[rng.choice(n_r, n_r // 4, replace=False)] = 999
    sk = s.key.copy()
    sk[:40] = 999
    p = hj.params("phj", 2, (6, 6), one_pass=True) if algo == "phj" else hj.params("shj", one_pass=True)
    tab = hj.Table(*to_dev(rk, r.rid), p=p)
    o_r, o_s, cnt = tab.probe(*to_dev(sk, s.rid))
    want_r, want_s = oracle.join(rk, r.rid, sk, s.rid)
    assert cnt == len(want_r)
    assert np.array_equal(canon(o_r, o_s), oracle.canonical(want_r, want_s))


def test_one_shot_batch():
    """hj_batch (plan, run once, free) gives every job the oracle's count and pairs."""
    specs = gen.batch_specs(49, 24, r_min=1024, r_max=1 << 16, max_factor=6)
    from paper_1307_1955_amd.gen import device as dgen
    jobs, want = [], []
    for sp in specs:
        rk, rr, sk, sr = dgen.job_relations(sp)
        cap = int((sk <= sp.n_r).sum().item())
        jobs.append((rk, rr, sk, sr, torch.empty(max(cap, 1), dtype=torch.int32, device=DEV)[:cap],
                     torch.empty(max(cap, 1), dtype=torch.int32, device=DEV)[:cap]))
        want.append(cap)
    d = torch.zeros(len(jobs), dtype=torch.int64, device=DEV)
    ws = torch.empty(hj.hj_batch_bytes(jobs, d), dtype=torch.uint8, device=DEV)
    hj.hj_batch(jobs, d, ws)
    assert d.cpu().tolist() == want
    for j in (0, len(jobs) // 2, len(jobs) - 1):
        rk, rr, sk, sr, o_r, o_s = jobs[j]
        w_r, w_s = oracle.join(*(x.cpu().numpy() for x in (rk, rr, sk, sr)))
        assert np.array_equal(canon(o_r, o_s), oracle.canonical(w_r, w_s))
