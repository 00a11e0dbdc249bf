"""GPU parity: the HIP join (through the C ABI) against the CPU oracle.

Results are integer pair multisets, so the bar is exact equality of the
canonical (sorted) forms.  Small cases span many tiles, partitions and work
items with ragged tails; full-size workloads are checked by closed forms on
every row plus the oracle on a sample of S rows.
"""
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


def to_dev(*arrays):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV) for a in arrays]


def gpu_join(p, rk, rr, sk, sr, capacity=None):
    o_r, o_s, cnt = hj.join(rk, rr, sk, sr, p=p, capacity=capacity)
    return o_r.cpu().numpy(), o_s.cpu().numpy(), cnt


def check_small(p, rk, rr, sk, sr):
    want_r, want_s = oracle.join(rk, rr, sk, sr)
    got_r, got_s, cnt = gpu_join(p, *to_dev(rk, rr, sk, sr))
    assert cnt == len(want_r), (cnt, len(want_r))
    assert np.array_equal(oracle.canonical(got_r, got_s), oracle.canonical(want_r, want_s))


def dup_relations(seed, n_r, n_s, domain):
    """Keys with duplicates on both sides, negative keys and int32 extremes."""
    rng = np.random.default_rng(seed)
    rk = rng.integers(-domain // 2, domain // 2, size=n_r).astype(np.int64)
    sk = rng.integers(-domain // 2, domain // 2 + domain // 4, size=n_s).astype(np.int64)
    ext = np.array([-(2 ** 31), 2 ** 31 - 1, 0, -1], dtype=np.int64)
    rk[: len(ext)] = ext
    sk[-len(ext):] = ext[::-1]
    rr = rng.permutation(n_r).astype(np.int32) * 3 + 1
    sr = rng.permutation(n_s).astype(np.int32) - 5
    return rk.astype(np.int32), rr, sk.astype(np.int32), sr


CASES = [
    ("shj", dict(algo="shj")),
    ("shj_1pass", dict(algo="shj", one_pass=True)),
    ("phj1_b1", dict(algo="phj", passes=1, bits=(1,))),
    ("phj1_b4", dict(algo="phj", passes=1, bits=(4,))),
    ("phj1_b8_t1024", dict(algo="phj", passes=1, bits=(8,), tile=1024)),
    ("phj1_b13_t8192", dict(algo="phj", passes=1, bits=(13,), tile=8192)),
    ("phj1_b10_t4096", dict(algo="phj", passes=1, bits=(10,), tile=4096)),
    ("phj2_2_3_t8192", dict(algo="phj", passes=2, bits=(2, 3), tile=8192)),
    ("phj2_6_6_t8192_1pass", dict(algo="phj", passes=2, bits=(6, 6), tile=8192, one_pass=True)),
    ("phj2_3_3", dict(algo="phj", passes=2, bits=(3, 3))),
    ("phj2_6_6", dict(algo="phj", passes=2, bits=(6, 6))),
    ("phj2_7_5_t2048", dict(algo="phj", passes=2, bits=(7, 5), tile=2048)),
    ("phj2_8_8", dict(algo="phj", passes=2, bits=(8, 8))),
    ("phj2_6_6_murmur", dict(algo="phj", passes=2, bits=(6, 6), hash="murmur2")),
    ("phj1_10_murmur", dict(algo="phj", passes=1, bits=(10,), hash="murmur2")),
    ("phj2_2_2_ldscap256", dict(algo="phj", passes=2, bits=(2, 2), lds_cap=256)),
    ("phj2_6_6_1pass", dict(algo="phj", passes=2, bits=(6, 6), one_pass=True)),
    ("phj1_3_1pass_ldscap256", dict(algo="phj", passes=1, bits=(3,), lds_cap=256, one_pass=True)),
    ("phj2_8_5_1pass_murmur", dict(algo="phj", passes=2, bits=(8, 5), hash="murmur2", one_pass=True)),
    # around the counted pass 2 (4..13 bits in all): 3 bits keep the pass-2
    # histogram; 12 and 9 bits in pass 2 reserve through LDS (more partitions per
    # segment than a wave has lanes) and 12 bits span several plan workgroups
    # per segment; small tiles run 256-thread workgroups; 1+7 bits with small
    # LDS tables have oversized partitions the scatter does not clear
    ("phj2_1_2", dict(algo="phj", passes=2, bits=(1, 2))),
    ("phj2_1_12_t4096", dict(algo="phj", passes=2, bits=(1, 12), tile=4096)),
    ("phj2_4_9_1pass", dict(algo="phj", passes=2, bits=(4, 9), one_pass=True)),
    ("phj2_5_5_t1024", dict(algo="phj", passes=2, bits=(5, 5), tile=1024)),
    ("phj2_1_7_ldscap256_1pass", dict(algo="phj", passes=2, bits=(1, 7), lds_cap=256, one_pass=True)),
]


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_small_duplicates(name, kw):
    rk, rr, sk, sr = dup_relations(1, 20011, 50021, 12000)
    check_small(hj.params(**kw), rk, rr, sk, sr)


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_small_unique_ragged(name, kw):
    r, s = gen.unique_uniform(5, 77777, 100003, 120000)
    check_small(hj.params(**kw), r.key, r.rid, s.key, s.rid)


@pytest.mark.parametrize("kw", [dict(algo="shj"), dict(algo="phj", passes=2, bits=(6, 6)),
                                dict(algo="phj", passes=1, bits=(5,))])
def test_empty_and_tiny(kw):
    p = hj.params(**kw)
    e = np.zeros(0, dtype=np.int32)
    one = np.array([42], dtype=np.int32)
    for rk, sk in [(e, e), (e, one), (one, e), (one, one), (one, -one)]:
        check_small(p, rk, np.arange(len(rk)), sk, np.arange(len(sk)) + 9)


@pytest.mark.parametrize("kw", [dict(algo="shj"), dict(algo="phj", passes=2, bits=(5, 5)),
                                dict(algo="phj", passes=2, bits=(5, 5), lds_cap=256),
                                dict(algo="shj", one_pass=True),
                                dict(algo="phj", passes=2, bits=(5, 5), lds_cap=256, one_pass=True)])
def test_cartesian_all_equal(kw):
    rk = np.full(300, 77, dtype=np.int32)
    sk = np.full(700, 77, dtype=np.int32)
    check_small(hj.params(**kw), rk, np.arange(300), sk, np.arange(700))


@pytest.mark.parametrize("kw", [dict(algo="shj"), dict(algo="phj", passes=2, bits=(6, 6)),
                                dict(algo="phj", passes=1, bits=(8,), hash="murmur2"),
                                dict(algo="phj", passes=2, bits=(6, 6), one_pass=True)])
@pytest.mark.parametrize("frac", [0.10, 0.25])
def test_r_side_skew(kw, frac):
    """A fraction of R shares one key (the low/high skew sets of Section 5.1): a heavy
    partition that overflows the LDS budget, and a many-to-many match."""
    n_r, n_s = 1 << 17, 1 << 18
    r, s = gen.unique_uniform(8, n_r, n_s, 2 * n_r)
    rk = r.key.copy()
    rng = np.random.default_rng(3)
    rk[rng.choice(n_r, int(n_r * frac), replace=False)] = 12345
    sk = s.key.copy()
    sk[:50] = 12345
    check_small(hj.params(**kw), rk, r.rid, sk, s.rid)


@pytest.mark.parametrize("kw", [dict(algo="phj", passes=2, bits=(4, 4), lds_cap=256),
                                dict(algo="phj", passes=2, bits=(4, 4), lds_cap=256, one_pass=True),
                                dict(algo="phj", passes=1, bits=(5,), one_pass=True),
                                dict(algo="shj"), dict(algo="shj", one_pass=True)])
def test_heavy_keys_hbm_path(kw):
    """Partitions beyond the LDS budget (identity hash: the partition is the key's low
    bits) with chains of very different length.  Partition 146 (mod 256) holds one key
    with 30000 R duplicates and 64 keys with 100 each, below that partition's heavy
    limit (r_len / 256), so those are walked; partition 239 holds a key with 3000
    duplicates and 16 keys with 100 each, all heavy there.  S matches them from many
    work items and rounds, 40 tuples of one key in one round (more than a round's
    heavy set holds).  For SHJ (one table over all 60001 rows, limit 234) the two
    big keys are heavy and the 100-long chains are walked."""
    rng = np.random.default_rng(21)
    n_r, n_s = 60001, 150001
    special = np.concatenate([np.full(30000, 4242), np.repeat((1 << 21) + 146 + 256 * np.arange(64), 100),
                              np.full(3000, -17), np.repeat((1 << 22) + 239 + 256 * np.arange(16), 100)])
    rk = np.concatenate([special, rng.integers(0, 1 << 20, size=n_r - len(special))]).astype(np.int32)
    rk = rk[rng.permutation(n_r)]
    sk = rng.integers(0, 1 << 20, size=n_s).astype(np.int32)
    sk[rng.choice(n_s, 60, replace=False)] = 4242
    sk[rng.choice(n_s, 500, replace=False)] = (1 << 21) + 146 + 256 * rng.integers(0, 64, size=500)
    sk[rng.choice(n_s, 200, replace=False)] = (1 << 22) + 239 + 256 * rng.integers(0, 16, size=200)
    sk[:40] = -17
    assert 4242 % 256 == 146 and (-17) % 256 == 239
    rr = rng.permutation(n_r).astype(np.int32)
    sr = rng.permutation(n_s).astype(np.int32) + 7
    check_small(hj.params(**kw), rk, rr, sk, sr)
    # a too-small output: the full count, only valid pairs below capacity, nothing past it
    want_r, want_s = oracle.join(rk, rr, sk, sr)
    want = len(want_r)
    cap = want // 2
    p = hj.params(**kw)
    buf_r = torch.full((want,), -9, dtype=torch.int32, device=DEV)
    buf_s = torch.full((want,), -9, dtype=torch.int32, device=DEV)
    ws = hj.workspace(p, n_r, n_s)
    d = torch.zeros(1, dtype=torch.int64, device=DEV)
    hj.hj_join(p, *to_dev(rk, rr, sk, sr), buf_r[:cap], buf_s[:cap], ws, d)
    torch.cuda.synchronize()
    assert int(d.item()) == want
    assert torch.all(buf_r[cap:] == -9) and torch.all(buf_s[cap:] == -9)
    got = oracle.canonical(buf_r[:cap].cpu().numpy(), buf_s[:cap].cpu().numpy())
    allp = oracle.canonical(want_r, want_s)
    # every written pair is a pair of the join, and no pair is written twice
    key = lambda a: a[:, 0].astype(np.int64) * (1 << 32) + a[:, 1].astype(np.int64) + (1 << 31)
    g, a = key(got), key(allp)
    assert len(np.unique(g)) == cap
    assert np.isin(g, a).all()


@pytest.mark.parametrize("kw", [dict(algo="shj"), dict(algo="shj", one_pass=True),
                                dict(algo="phj", passes=2, bits=(4, 4), lds_cap=256, one_pass=True),
                                dict(algo="phj", passes=1, bits=(3,))])
def test_interleaved_heavy_keys(kw):
    """Several heavy keys interleaved row by row (runs onto different slots inside
    one wave, pending chains flushed and restarted at every row), among them the
    int32 extremes and -1 (the empty slot's key bits), plus unique keys; S hits
    each heavy key a few times."""
    n_r, n_s = 50000, 90001
    heavy = np.array([-1, -(2 ** 31), 2 ** 31 - 1, 7, 7 + 8, 7 + 16], dtype=np.int64)
    rk = np.arange(n_r, dtype=np.int64) * 64 + 1000          # unique keys, outside the heavy set
    rows = np.arange(0, 36000)
    rk[rows] = heavy[rows % len(heavy)]                       # 6000 rows per heavy key, interleaved
    rng = np.random.default_rng(23)
    sk = rng.integers(0, n_r * 64 + 1000, size=n_s)
    for i, k in enumerate(heavy):
        sk[rng.choice(n_s, 3, replace=False)] = k
    rr = rng.permutation(n_r).astype(np.int32)
    sr = rng.permutation(n_s).astype(np.int32)
    check_small(hj.params(**kw), rk.astype(np.int32), rr, sk.astype(np.int32), sr)


@pytest.mark.parametrize("one_pass", [True, False])
def test_shj_heavy_queue_overflow(one_pass):
    """One-pass SHJ hands heavy S tuples to a 256-entry queue that every workgroup
    helps with; here 400 S tuples hit one heavy key of an R spanning several 64K-row
    chunks, so the queue fills and the rest stay with their workgroups' own scans
    (two-pass SHJ: all of them block-local).  Every pair against the oracle."""
    n_r, n_s = 150001, 200003
    rng = np.random.default_rng(29)
    rk = rng.permutation(n_r).astype(np.int64) + 1
    rk[rng.choice(n_r, 15000, replace=False)] = 77
    sk = rng.integers(1, 2 * n_r, size=n_s)
    sk[rng.choice(n_s, 400, replace=False)] = 77
    rr = rng.permutation(n_r).astype(np.int32)
    sr = rng.permutation(n_s).astype(np.int32)
    check_small(hj.params("shj", one_pass=one_pass), rk.astype(np.int32), rr, sk.astype(np.int32), sr)


@pytest.mark.parametrize("kw", [dict(algo="phj", passes=2, bits=(6, 6), one_pass=True),
                                dict(algo="phj", passes=1, bits=(8,), one_pass=True),
                                dict(algo="phj", passes=2, bits=(6, 6))], ids=["6_6_1pass", "8_1pass", "6_6"])
@pytest.mark.parametrize("n_heavy_s", [40, 300])
def test_phj_heavy_queue(kw, n_heavy_s):
    """One-pass PHJ hands the heavy S tuples of an HBM-table partition larger than
    one 64K-row chunk (70000 R rows on key 77) to the device-wide queue every
    workgroup helps with; 300 such tuples overflow its 256 entries and the rest
    stay with their workgroups' own scans.  Two-pass output keeps the
    workgroup-local scans.  Every pair against the oracle."""
    n_r, n_s = 1 << 19, 1 << 20
    r, s = gen.unique_uniform(33, n_r, n_s, 2 * n_r)
    rng = np.random.default_rng(34)
    rk = r.key.copy()
    rk[rng.choice(n_r, 70000, replace=False)] = 77
    sk = s.key.copy()
    sk[rng.choice(n_s, n_heavy_s, replace=False)] = 77
    check_small(hj.params(**kw), rk, r.rid, sk, s.rid)


@pytest.mark.parametrize("kw", [dict(algo="phj", passes=1, bits=(6,), one_pass=True),
                                dict(algo="phj", passes=2, bits=(3, 3), one_pass=True),
                                dict(algo="phj", passes=2, bits=(3, 3), one_pass=False)],
                         ids=["6_1pass", "3_3_1pass", "3_3"])
def test_phj_heavy_queue_many_partitions(kw):
    """Four keys with 70000 R rows each, in four different partitions (identity
    hash: the key's low bits), so the overflow build flags four partitions and
    sums their work items for the write's helpers to wait on; S tuples hit
    three of the keys (the fourth partition is flagged but queues nothing).
    Every pair against the oracle."""
    n_r, n_s = 1 << 20, 1 << 21
    r, s = gen.unique_uniform(35, n_r, n_s, 2 * n_r)
    rng = np.random.default_rng(36)
    rk = r.key.copy()
    keys = [77, 78, 79, 80]  # partitions 13, 14, 15, 16 of 64
    rows = rng.permutation(n_r)[: 4 * 70000].reshape(4, 70000)
    for k, rw in zip(keys, rows):
        rk[rw] = k
    sk = s.key.copy()
    for k in keys[:3]:
        sk[rng.choice(n_s, 25, replace=False)] = k
    check_small(hj.params(**kw), rk, r.rid, sk, s.rid)


@pytest.mark.parametrize("one_pass", [True, False])
def test_sorted_r_short_duplicate_runs(one_pass):
    """R sorted with 32 duplicates per key: every build wave pushes runs of 32 rows
    onto one slot, so up to 63 keys are recorded as hot, yet every chain (32 rows)
    is far below the heavy limit.  A probe registers a hot key's tuple at once only
    when the recorded rows exceed its walk limit; here the walks decide, and the
    result is the same multiset either way."""
    n_r, n_s = 1 << 18, 1 << 18
    rng = np.random.default_rng(61)
    rk = (np.arange(n_r, dtype=np.int64) // 32).astype(np.int32)
    sk = rng.integers(-100, n_r // 32 + 100, size=n_s).astype(np.int32)
    rr = np.arange(n_r, dtype=np.int32)
    sr = rng.permutation(n_s).astype(np.int32)
    check_small(hj.params("shj", one_pass=one_pass), rk, rr, sk, sr)


def offset_view(a, off):
    """Device copy of `a` that starts `off` int32 elements into a larger buffer
    (input columns at every 4-byte alignment inside a 16-byte line)."""
    buf = torch.zeros(len(a) + 8, dtype=torch.int32, device=DEV)
    buf[off: off + len(a)] = torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)
    return buf[off: off + len(a)]


@pytest.mark.parametrize("offs", [(1, 1, 3, 3), (1, 2, 0, 3), (3, 0, 2, 2)])
@pytest.mark.parametrize("kw", [dict(algo="phj", passes=2, bits=(6, 6)), dict(algo="phj", passes=1, bits=(7,)),
                                dict(algo="phj", passes=2, bits=(5, 4), one_pass=True, tile=1024),
                                dict(algo="phj", passes=2, bits=(6, 5), tile=8192),
                                dict(algo="shj")])
def test_misaligned_columns(kw, offs):
    """Key and rid columns at different offsets inside 16-byte lines (vector and
    element-wise tile loads), ragged sizes."""
    rk, rr, sk, sr = dup_relations(12, 70001, 130003, 90000)
    cols = [offset_view(a, o) for a, o in zip((rk, rr, sk, sr), offs)]
    want_r, want_s = oracle.join(rk, rr, sk, sr)
    o_r, o_s, cnt = hj.join(*cols, p=hj.params(**kw))
    assert cnt == len(want_r)
    assert np.array_equal(oracle.canonical(o_r.cpu().numpy(), o_s.cpu().numpy()), oracle.canonical(want_r, want_s))


@pytest.mark.parametrize("kw", [dict(algo="shj"), dict(algo="phj", passes=2, bits=(6, 6)),
                                dict(algo="phj", passes=1, bits=(3,)),
                                dict(algo="phj", passes=2, bits=(6, 6), one_pass=True),
                                dict(algo="shj", one_pass=True)])
def test_capacity_guard(kw):
    """Too small an output: the full count is reported, nothing is written past capacity."""
    p = hj.params(**kw)
    r, s = gen.unique_uniform(9, 30000, 60000, 40000)
    rk, rr, sk, sr = to_dev(r.key, r.rid, s.key, s.rid)
    want = oracle.join_count(r.key, r.rid, s.key)
    cap = want // 3
    buf_r = torch.full((want,), -7, dtype=torch.int32, device=DEV)
    buf_s = torch.full((want,), -7, dtype=torch.int32, device=DEV)
    ws = hj.workspace(p, len(r), len(s))
    d_count = torch.zeros(1, dtype=torch.int64, device=DEV)
    with pytest.raises(hj.HJError) as e:
        hj.hj_join_sync(p, rk, rr, sk, sr, buf_r[:cap], buf_s[:cap], ws, d_count)
    assert e.value.status == hj.HJ_ERR_CAPACITY
    assert int(d_count.item()) == want
    assert torch.all(buf_r[cap:] == -7) and torch.all(buf_s[cap:] == -7)
    # the asynchronous call reports the count in device memory as well
    d_count.zero_()
    hj.hj_join(p, rk, rr, sk, sr, buf_r[:0], buf_s[:0], ws, d_count)
    torch.cuda.synchronize()
    assert int(d_count.item()) == want


def test_repeatable_and_timed():
    p = hj.params("phj", 2, (6, 6))
    r, s = gen.unique_uniform(4, 1 << 16, 1 << 17, 1 << 17)
    t = to_dev(r.key, r.rid, s.key, s.rid)
    a = gen_canon(p, t)
    b = gen_canon(p, t)
    assert np.array_equal(a, b)
    out_r = torch.empty(len(s), dtype=torch.int32, device=DEV)
    out_s = torch.empty(len(s), dtype=torch.int32, device=DEV)
    ws = hj.workspace(p, len(r), len(s))
    d_count = torch.zeros(1, dtype=torch.int64, device=DEV)
    launches = hj.hj_join_timed(p, *t, out_r, out_s, ws, d_count)
    names = [n for n, _ in launches]
    assert "part_scatter" in names and "join_write" in names
    assert all(ms >= 0 for _, ms in launches)
    cnt = int(d_count.item())
    assert np.array_equal(oracle.canonical(out_r[:cnt].cpu().numpy(), out_s[:cnt].cpu().numpy()), a)


def gen_canon(p, t):
    o_r, o_s, cnt = hj.join(*t, p=p)
    return oracle.canonical(o_r.cpu().numpy(), o_s.cpu().numpy())


# ---------------------------------------------------------------------------
# Device generator == host generator (so device-made inputs are the generator's)
# ---------------------------------------------------------------------------


def test_device_generator_matches_host():
    rng = np.random.default_rng(0)
    n = (1 << 20) + 17
    idx = rng.integers(0, n, size=5000)
    pk = dgen.perm_keys(3, 1, n).cpu().numpy()
    assert np.array_equal(pk[idx], gen.permutation_at(3, 1, n, idx) + 1)
    assert np.array_equal(np.sort(pk), np.arange(1, n + 1))
    uk = dgen.uniform_keys(3, 2, n, 999983).cpu().numpy()
    assert np.array_equal(uk[idx], gen.uniform_int_at(3, 2, idx, 1, 999983))
    cdf = gen.zipf_cdf(1 << 16, 1.0)
    zk = dgen.zipf_keys(3, 2, n, torch.from_numpy(cdf).to(DEV)).cpu().numpy()
    assert np.array_equal(zk[idx], gen.zipf_ranks_at(3, 2, idx, cdf))
    r_host, s_host = gen.config_c1(seed=1, n=1 << 16)
    rk, rr, sk, sr = dgen.config_c1(seed=1, n=1 << 16)
    assert np.array_equal(rk.cpu().numpy(), r_host.key) and np.array_equal(sk.cpu().numpy(), s_host.key)
    assert np.array_equal(rr.cpu().numpy(), r_host.rid) and np.array_equal(sr.cpu().numpy(), s_host.rid)
    r_host, s_host = gen.skewed_r(4, 1 << 16, 1 << 17, 1 << 17, 0.25)
    rk, rr, sk, sr = dgen.skewed_r(4, 1 << 16, 1 << 17, 1 << 17, 0.25)
    assert np.array_equal(rk.cpu().numpy(), r_host.key) and np.array_equal(sk.cpu().numpy(), s_host.key)


# ---------------------------------------------------------------------------
# Full-size workloads
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("frac", [0.10, 0.25])
def test_paper_skew_sets_16m(frac):
    """Section 5.1's low- and high-skew sets at 16M x 16M (R: a fraction frac of the
    rows on one key, S uniform over 1..2^25), with three S tuples forced onto the
    skewed key so the probe meets its chain: PHJ (library choice) and SHJ, every
    pair against the oracle (one-pass SHJ hands the heavy tuples to the device-wide
    queue that every workgroup helps with)."""
    n = 1 << 24
    r, s = gen.skewed_r(31, n, n, 2 * n, frac)
    s.key[[5, n // 2, n - 1]] = gen.SKEW_KEY
    want_r, want_s = oracle.join(r.key, r.rid, s.key, s.rid)
    want = oracle.canonical(want_r, want_s)
    del want_r, want_s
    t = to_dev(r.key, r.rid, s.key, s.rid)
    for p in (hj.params("auto", one_pass=True), hj.params("shj"), hj.params("shj", one_pass=True)):
        got_r, got_s, cnt = gpu_join(p, *t, capacity=len(want))
        assert cnt == len(want)
        assert np.array_equal(oracle.canonical(got_r, got_s), want)


def closed_form_unique(r_key, s_key):
    n = len(r_key)
    inv = np.empty(n + 1, dtype=np.int64)
    inv[r_key.astype(np.int64)] = np.arange(n)
    m = np.full(len(s_key), -1, dtype=np.int64)
    hit = s_key.astype(np.int64) <= n
    m[hit] = inv[s_key[hit].astype(np.int64)]
    return m


def check_full(p, rk, rr, sk, sr, seed, sample=1 << 16):
    """Every row against the closed form; a sample of S rows against the oracle;
    sampled rows of the device-made input against the host generator."""
    o_r, o_s, cnt = hj.join(rk, rr, sk, sr, p=p)
    r_key, s_key = rk.cpu().numpy(), sk.cpu().numpy()
    m = oracle.match_of(o_r.cpu().numpy(), o_s.cpu().numpy(), len(s_key))
    expect = closed_form_unique(r_key, s_key)
    assert cnt == int(np.sum(expect >= 0))
    assert np.array_equal(m, expect)
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(len(s_key), size=min(sample, len(s_key)), replace=False))
    w_r, w_s = oracle.join(r_key, np.arange(len(r_key)), s_key[rows], rows)
    got = np.stack([m[rows], rows], axis=1)
    got = got[got[:, 0] >= 0]
    assert np.array_equal(oracle.canonical(got[:, 0], got[:, 1]), oracle.canonical(w_r, w_s))
    return r_key, s_key, rows


C1_C2_PARAMS = [
    ("shj", dict(algo="shj")),
    ("phj2_6_6", dict(algo="phj", passes=2, bits=(6, 6))),
    ("phj1_12", dict(algo="phj", passes=1, bits=(12,))),
    ("phj2_7_6_murmur", dict(algo="phj", passes=2, bits=(7, 6), hash="murmur2")),
    ("phj2_6_6_1pass", dict(algo="phj", passes=2, bits=(6, 6), one_pass=True)),
    ("shj_1pass", dict(algo="shj", one_pass=True)),
    # counted pass 2 with more partitions per segment than a wave has lanes
    ("phj2_5_8_1pass", dict(algo="phj", passes=2, bits=(5, 8), one_pass=True)),
    ("phj2_6_7", dict(algo="phj", passes=2, bits=(6, 7))),
]


@pytest.mark.parametrize("name,kw", C1_C2_PARAMS, ids=[c[0] for c in C1_C2_PARAMS])
def test_c1_full_vs_oracle(name, kw):
    """1M x 1M, every S tuple matches once: compared in full with the oracle."""
    r, s = gen.config_c1()
    want = oracle.match_of(*oracle.join(r.key, r.rid, s.key, s.rid), len(s))
    o_r, o_s, cnt = hj.join(*to_dev(r.key, r.rid, s.key, s.rid), p=hj.params(**kw))
    assert cnt == 1 << 20
    assert np.array_equal(oracle.match_of(o_r.cpu().numpy(), o_s.cpu().numpy(), len(s)), want)


@pytest.mark.parametrize("name,kw", C1_C2_PARAMS, ids=[c[0] for c in C1_C2_PARAMS])
def test_c2_full(name, kw):
    """16M x 16M, about half of S matches."""
    rk, rr, sk, sr = dgen.config_c2()
    r_key, s_key, rows = check_full(hj.params(**kw), rk, rr, sk, sr, seed=2)
    assert np.array_equal(r_key[rows[:1000] % len(r_key)],
                          gen.permutation_at(2, gen.STREAM_R_KEYS, 1 << 24, rows[:1000] % len(r_key)) + 1)
    assert np.array_equal(s_key[rows], gen.uniform_int_at(2, gen.STREAM_S_KEYS, rows, 1, 1 << 25))


# 16M x 16M in one pass of few radix bits (and 7 + 7): every R partition is
# larger than the LDS table and joins through the HBM-table path.  With the
# identity hash the partitions are exactly equal (1024 build items of 16384 R
# tuples); MurmurHash 2.0 makes them uneven, so there are more build items than
# the 1024 workgroups of the HBM-table launches and their grid-stride loops turn.
C2_WIDE_PARAMS = [
    ("phj1_6", dict(algo="phj", passes=1, bits=(6,))),
    ("phj1_6_murmur_1pass", dict(algo="phj", passes=1, bits=(6,), hash="murmur2", one_pass=True)),
    ("phj1_7_1pass", dict(algo="phj", passes=1, bits=(7,), one_pass=True)),
    ("phj1_8_murmur", dict(algo="phj", passes=1, bits=(8,), hash="murmur2")),
    ("phj1_10_murmur_1pass", dict(algo="phj", passes=1, bits=(10,), hash="murmur2", one_pass=True)),
    ("phj1_10", dict(algo="phj", passes=1, bits=(10,))),
    ("phj2_7_7", dict(algo="phj", passes=2, bits=(7, 7))),
    ("phj2_7_7_1pass", dict(algo="phj", passes=2, bits=(7, 7), one_pass=True)),
]


def murmur2_np(k):
    """MurmurHash 2.0 of each 4-byte key (the radix hash HJ_HASH_MURMUR2), in
    numpy, to count the partitions a configuration makes."""
    m = np.uint64(0x5bd1e995)
    mask = np.uint64(0xFFFFFFFF)
    k = k.astype(np.uint32).astype(np.uint64)
    h = (np.uint64(0x9747b28c) ^ np.uint64(4)) & mask
    k = (k * m) & mask
    k ^= k >> np.uint64(24)
    k = (k * m) & mask
    h = (h * m) & mask
    h ^= k
    h ^= h >> np.uint64(13)
    h = (h * m) & mask
    h ^= h >> np.uint64(15)
    return h.astype(np.uint32)


def hbm_build_items(p, r_key, s_key):
    """HBM-table build items of a one-pass configuration: ceil(|R_i| / 16384) for
    every partition with |R_i| above the LDS table and a non-empty S_i."""
    q = hj.hj_resolve_params(p, len(r_key), len(s_key))
    B = q.bits[0] + (q.bits[1] if q.passes == 2 else 0)
    f = murmur2_np if q.hash == hj.HJ_HASH_MURMUR2 else (lambda a: a.astype(np.uint32))
    mask = np.uint32((1 << B) - 1)
    r_len = np.bincount(f(r_key) & mask, minlength=1 << B)
    s_len = np.bincount(f(s_key) & mask, minlength=1 << B)
    big = (r_len > q.lds_cap) & (s_len > 0)
    return int(np.sum((r_len[big] + 16383) // 16384))


@pytest.mark.parametrize("name,kw", C2_WIDE_PARAMS, ids=[c[0] for c in C2_WIDE_PARAMS])
def test_c2_full_hbm_tables(name, kw):
    """16M x 16M through the HBM-table path for every partition: every row against
    the closed form, a sample of S rows against the oracle."""
    rk, rr, sk, sr = dgen.config_c2()
    p = hj.params(**kw)
    r_key, s_key, rows = check_full(p, rk, rr, sk, sr, seed=22)
    if kw["passes"] == 1:
        items = hbm_build_items(p, r_key, s_key)
        if kw.get("hash") == "murmur2":
            assert items > 1024, items  # the build launches' grid-stride loops run a second time
        else:
            assert items == 1024, items


# Joins of 2^24 tuples and more read their partitioning tiles (and, while
# |S| <= 2 |R|, the join's S chunks) with non-temporal loads, and SHJ builds of
# |R| >= 2^23 their R keys: the shapes on both sides of those thresholds, each
# kernel variant in both output modes, every row against the closed form.
NT_SHAPES = [
    ("2m_16m_phj1_9", 1 << 21, 1 << 24, dict(algo="phj", passes=1, bits=(9,), tile=8192, one_pass=True)),
    ("2m_16m_phj2_4_5", 1 << 21, 1 << 24, dict(algo="phj", passes=2, bits=(4, 5))),
    ("8m_16m_phj2_5_6_1pass", 1 << 23, 1 << 24, dict(algo="phj", passes=2, bits=(5, 6), tile=4096, one_pass=True)),
    ("8m_16m_phj2_5_6", 1 << 23, 1 << 24, dict(algo="phj", passes=2, bits=(5, 6), tile=4096)),
    ("8m_8m_phj2_5_6_1pass", 1 << 23, 1 << 23, dict(algo="phj", passes=2, bits=(5, 6), one_pass=True)),
    ("8m_8m_shj_1pass", 1 << 23, 1 << 23, dict(algo="shj", one_pass=True)),
    ("4m_8m_shj", 1 << 22, 1 << 23, dict(algo="shj")),
]


@pytest.mark.parametrize("name,n_r,n_s,kw", NT_SHAPES, ids=[c[0] for c in NT_SHAPES])
def test_non_temporal_shapes(name, n_r, n_s, kw):
    """Every row against the closed form, a sample of S rows against the oracle."""
    rk, rr, sk, sr = dgen.unique_uniform(31, n_r, n_s, 2 * n_r, "cuda")
    check_full(hj.params(**kw), rk, rr, sk, sr, seed=31)


@pytest.mark.parametrize("theta", [0.5, 1.0])
@pytest.mark.parametrize("kw", [dict(algo="phj", passes=2, bits=(6, 6)), dict(algo="shj"),
                                dict(algo="phj", passes=2, bits=(6, 6), one_pass=True)],
                         ids=["phj2_6_6", "shj", "phj2_6_6_1pass"])
def test_c3_zipf_full(theta, kw):
    """16M R, 64M Zipf S: every S tuple matches; heavy hitters split over many work items."""
    rk, rr, sk, sr = dgen.config_c3(theta=theta)
    r_key, s_key, rows = check_full(hj.params(**kw), rk, rr, sk, sr, seed=3)
    cdf = gen.zipf_cdf(1 << 24, theta)
    assert np.array_equal(s_key[rows[:2000]], gen.zipf_ranks_at(3, gen.STREAM_S_KEYS, rows[:2000], cdf))


@pytest.mark.parametrize("n_r,n_s,bits", [(1 << 21, 1 << 24, 9), (1 << 22, (1 << 24) - (1 << 22), 10)])
def test_one_pass_wide(n_r, n_s, bits):
    """One pass of 9 and 10 radix bits with 8192-tuple tiles in 512-thread
    workgroups (partitions of 4096 R tuples): every S row against the closed
    form, a sample of S rows against the oracle."""
    p = hj.params("phj", 1, (bits,), tile=8192, one_pass=True)
    q = hj.hj_resolve_params(p, n_r, n_s)
    assert q.passes == 1 and q.bits[0] == bits and q.tile == 8192
    rk, rr, sk, sr = dgen.unique_uniform(50, n_r, n_s, 2 * n_r)
    o_r, o_s, cnt = hj.join(rk, rr, sk, sr, p=p)
    s_key = sk.cpu().numpy()
    assert cnt == int((s_key <= n_r).sum())
    m = oracle.match_of(o_r.cpu().numpy(), o_s.cpu().numpy(), n_s)
    r_key = rk.cpu().numpy()
    inv = np.empty(n_r + 1, dtype=np.int64)
    inv[r_key.astype(np.int64)] = np.arange(n_r)
    want = np.where(s_key <= n_r, inv[np.minimum(s_key, n_r).astype(np.int64)], -1)
    assert np.array_equal(m, want)
    rows = np.sort(np.random.default_rng(51).choice(n_s, size=1 << 15, replace=False))
    w_r, w_s = oracle.join(r_key, np.arange(n_r, dtype=np.int32), s_key[rows], rows.astype(np.int32))
    got = np.stack([m[rows], rows], axis=1)
    got = got[got[:, 0] >= 0]
    assert np.array_equal(oracle.canonical(got[:, 0], got[:, 1]), oracle.canonical(w_r, w_s))
