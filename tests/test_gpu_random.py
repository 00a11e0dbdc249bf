"""Seeded random sweep over the parameter space (algorithm, passes, radix bits,
tile, hash, LDS capacity, output mode) and input shapes (sizes from empty to a
few hundred thousand, key domains from all-duplicate to unique): every join,
through hj_join and through hj_build + hj_probe, equals the oracle's pair
multiset.  Deterministic: the cases come from fixed seeds."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1307_1955_amd.hj as hj  # noqa: E402

DEV = torch.device("cuda:0")
NCASES = 48


def random_case(seed):
    rng = np.random.default_rng(1000 + seed)
    n_r = 0 if rng.random() < 0.05 else int(np.exp(rng.uniform(0, np.log(200000))))
    n_s = 0 if rng.random() < 0.05 else int(np.exp(rng.uniform(0, np.log(300000))))
    domain = max(1, int(np.exp(rng.uniform(0, np.log(4 * max(n_r, 1) + 1)))))
    lo = int(rng.integers(-(2 ** 31), 2 ** 31 - domain))
    rk = (lo + rng.integers(0, domain, size=n_r)).astype(np.int32)
    sk = (lo + rng.integers(0, domain + domain // 3 + 1, size=n_s)).astype(np.int32)
    rr = rng.permutation(n_r).astype(np.int32) - 3
    sr = (rng.permutation(n_s) * 2).astype(np.int32)
    algo = rng.choice(["shj", "phj", "phj", "auto"])
    kw = dict(algo=str(algo), one_pass=bool(rng.random() < 0.5), hash=str(rng.choice(["identity", "murmur2"])),
              tile=int(rng.choice([0, 1024, 2048, 4096, 8192])))
    if algo == "phj":
        passes = int(rng.choice([0, 1, 2])) if n_r <= 8192 else int(rng.choice([1, 2]))
        kw["passes"] = passes
        if passes == 1:
            kw["bits"] = (int(rng.integers(1, 14)),)
        elif passes == 2:
            b1 = int(rng.integers(1, 14))
            kw["bits"] = (b1, int(rng.integers(1, min(13, 16 - b1) + 1)))
        else:
            kw["bits"] = (0, 0)
        if rng.random() < 0.3:
            need = 64 * ((n_r + 63) // 64) if passes == 0 else 256
            kw["lds_cap"] = int(64 * rng.integers(max(4, need // 64), 129))
    return rk, rr, sk, sr, kw


@pytest.mark.parametrize("seed", range(NCASES))
def test_random_join(seed):
    rk, rr, sk, sr, kw = random_case(seed)
    p = hj.params(**kw)
    want = oracle.canonical(*oracle.join(rk, rr, sk, sr))
    t = [torch.from_numpy(a).to(DEV) for a in (rk, rr, sk, sr)]
    o_r, o_s, cnt = hj.join(*t, p=p)
    assert cnt == len(want), (kw, len(rk), len(sk))
    assert np.array_equal(oracle.canonical(o_r.cpu().numpy(), o_s.cpu().numpy()), want), kw
    if seed % 2 == 0:  # the split join on the same inputs
        tab = hj.Table(t[0], t[1], p=p)
        b_r, b_s, bcnt = tab.probe(t[2], t[3])
        assert bcnt == len(want), kw
        assert np.array_equal(oracle.canonical(b_r.cpu().numpy(), b_s.cpu().numpy()), want), kw
