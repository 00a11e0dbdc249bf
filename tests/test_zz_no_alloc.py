"""hj_join_noalloc (the join on the library's fixed device workspace, for callers
that cannot allocate) against hj_join with a caller workspace: the same pair
multiset and count, bit for bit, on two calls in a row with the second one
smaller (the fixed array keeps the first call's contents), for SHJ, PHJ with
one and two radix passes and both output modes, and the direct LDS join."""
import ctypes

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


def relations(seed, n_r, n_s, dups):
    r, s = gen.unique_uniform(seed, n_r, n_s, 2 * n_r)
    rk = r.key.copy()
    if dups:  # duplicates on both sides
        k = n_r // 8
        rk[:k] = rk[k: 2 * k]
    return [torch.from_numpy(a).to(DEV) for a in (rk, r.rid, s.key, s.rid)]


def with_workspace(p, t):
    o_r, o_s, cnt = hj.join(*t, p=p)
    return oracle.canonical(o_r.cpu().numpy(), o_s.cpu().numpy()), cnt


def noalloc(p, t, cap):
    o_r = torch.full((max(cap, 1),), -3, dtype=torch.int32, device=DEV)
    o_s = torch.full((max(cap, 1),), -3, dtype=torch.int32, device=DEV)
    d = torch.zeros(1, dtype=torch.int64, device=DEV)
    R = hj._rel(t[0], t[1], "R")
    S = hj._rel(t[2], t[3], "S")
    O = hj._out(o_r[:cap], o_s[:cap])
    st = hj.load().hj_join_noalloc(ctypes.byref(p), ctypes.byref(R), ctypes.byref(S), ctypes.byref(O),
                                   d.data_ptr(), hj._stream(None))
    assert st == hj.HJ_OK, hj.load().hj_last_error()
    torch.cuda.synchronize()
    cnt = int(d.item())
    assert cnt <= cap
    return oracle.canonical(o_r[:cnt].cpu().numpy(), o_s[:cnt].cpu().numpy()), cnt


CASES = [
    ("shj", dict(algo="shj")),
    ("shj_1pass", dict(algo="shj", one_pass=True)),
    ("phj2_6_6", dict(algo="phj", passes=2, bits=(6, 6))),
    ("phj2_5_4_1pass", dict(algo="phj", passes=2, bits=(5, 4), one_pass=True)),
    ("phj1_8", dict(algo="phj", passes=1, bits=(8,))),
    ("auto_1pass", dict(algo="auto", one_pass=True)),
]


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_hj_join(name, kw):
    p = hj.params(**kw)
    for i, (n_r, n_s) in enumerate([(600_000, 1_000_003), (70_001, 150_007)]):  # second call smaller
        t = relations(70 + i, n_r, n_s, dups=(i == 1))
        want, cnt = with_workspace(p, t)
        got, cnt2 = noalloc(p, t, cnt + 100)
        assert cnt2 == cnt
        assert np.array_equal(got, want)


def test_noalloc_direct_then_smaller():
    p = hj.params("phj", passes=0)
    for i, (n_r, n_s) in enumerate([(8000, 400_000), (300, 5_000)]):
        t = relations(80 + i, n_r, n_s, dups=True)
        want, cnt = with_workspace(p, t)
        got, cnt2 = noalloc(p, t, cnt)
        assert cnt2 == cnt and np.array_equal(got, want)


def test_noalloc_rejects_beyond_its_workspace():
    p = hj.params("phj", 2, (6, 6))
    R = hj.HjRel(256, 256, 1 << 24)
    S = hj.HjRel(256, 256, 1 << 24)
    O = hj.HjOut(256, 256, 1 << 24)
    lib = hj.load()
    assert lib.hj_join_noalloc(ctypes.byref(p), ctypes.byref(R), ctypes.byref(S), ctypes.byref(O), 256,
                               None) == hj.HJ_ERR_WORKSPACE
    assert b"fixed" in lib.hj_last_error()
