"""GPU tests of the join server: every result is the same alone and in the mix
of overlapping requests, admission respects the memory cap, and footprints
are released when requests finish."""
import time

import numpy as np
import pytest

import oracle
from paper_1307_1955_amd import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1307_1955_amd.hj as hj  # noqa: E402
from paper_1307_1955_amd import tune  # noqa: E402
from paper_1307_1955_amd.gen import device as dgen  # noqa: E402

DEV = torch.device("cuda:0")


def requests(seed, n, r_max=1 << 17):
    specs = gen.batch_specs(seed, n, r_min=1024, r_max=r_max, max_factor=8)
    reqs = []
    table = tune.load_table()
    for sp in specs:
        rk, rr, sk, sr = dgen.job_relations(sp)
        cap = int((sk <= sp.n_r).sum().item())
        o_r = torch.full((max(cap, 1),), -1, dtype=torch.int32, device=DEV)
        o_s = torch.full((max(cap, 1),), -1, dtype=torch.int32, device=DEV)
        p = tune.choose(sp.n_r, sp.n_s, table).params()
        # the server's own account: relations, output slots, the count, the workspace
        fp = 8 * (sp.n_r + sp.n_s) + 8 * cap + 8 + hj.hj_workspace_bytes(p, sp.n_r, sp.n_s)
        reqs.append(dict(spec=sp, t=[rk, rr, sk, sr, o_r[:cap], o_s[:cap]], cap=cap, p=p, fp=fp))
    return reqs


def test_results_same_alone_and_in_mix():
    reqs = requests(21, 48)
    counts = torch.zeros(len(reqs), dtype=torch.int64, device=DEV)
    ws = torch.empty(1 << 30, dtype=torch.uint8, device=DEV)
    sv = hj.Server(ws, mem_cap_bytes=64 << 30, slots=4, max_batch_jobs=8)
    tickets = {}
    for i, r in enumerate(reqs):
        tickets[sv.submit(*r["t"], counts[i:i + 1], r["p"], r["fp"])] = i
        if i % 7 == 0:
            time.sleep(0.0005)  # arrivals spread over time, so later ones join running batches
    sv.drain()
    done = sv.poll()
    assert sorted(t for t, *_ in done) == sorted(tickets)
    assert all(st == hj.HJ_OK for _, st, _, _ in done)
    st = sv.stats()
    assert st["completed"] == len(reqs) and st["rejected"] == 0 and st["bytes_in_use"] == 0
    assert st["batches"] >= 2
    sv.close()
    got_counts = counts.cpu().numpy()
    for i, r in enumerate(reqs):
        c = int(got_counts[i])
        assert c == r["cap"]
        mix = oracle.canonical(r["t"][4][:c].cpu().numpy(), r["t"][5][:c].cpu().numpy())
        a_r, a_s, a_c = hj.join(*r["t"][:4], p=r["p"])
        assert a_c == c
        alone = oracle.canonical(a_r.cpu().numpy(), a_s.cpu().numpy())
        assert np.array_equal(mix, alone), i
        if i % 6 == 0:  # and against the oracle
            rk, rr, sk, sr = (x.cpu().numpy() for x in r["t"][:4])
            w_r, w_s = oracle.join(rk, rr, sk, sr)
            assert np.array_equal(mix, oracle.canonical(w_r, w_s)), i


def test_admission_cap_and_rejection():
    reqs = requests(22, 12)
    counts = torch.zeros(len(reqs), dtype=torch.int64, device=DEV)
    ws = torch.empty(1 << 30, dtype=torch.uint8, device=DEV)
    big = max(r["fp"] for r in reqs)
    cap = big + 1  # only about one request fits at a time
    sv = hj.Server(ws, mem_cap_bytes=cap, slots=4, max_batch_jobs=16)
    for i, r in enumerate(reqs):
        sv.submit(*r["t"], counts[i:i + 1], r["p"], r["fp"])
    # one request larger than the cap is rejected
    huge = reqs[0]
    t_rej = sv.submit(*huge["t"], counts[0:1], huge["p"], cap + 1)
    sv.drain()
    done = {t: (s, lat, q) for t, s, lat, q in sv.poll()}
    assert done[t_rej][0] == hj.HJ_ERR_CAPACITY
    ok = [t for t, v in done.items() if v[0] == hj.HJ_OK]
    assert len(ok) == len(reqs)
    st = sv.stats()
    assert st["rejected"] == 1 and st["bytes_in_use"] == 0
    sv.close()
    got = counts.cpu().numpy()
    for i, r in enumerate(reqs[1:], start=1):
        assert int(got[i]) == r["cap"]


def test_footprint_floor():
    """A request declared smaller than its own arrays and workspace is admitted by
    the server's account of it: rejected under a cap below that account, run
    under a cap at it."""
    reqs = requests(23, 2)
    r = reqs[1]
    counts = torch.zeros(2, dtype=torch.int64, device=DEV)
    ws = torch.empty(1 << 28, dtype=torch.uint8, device=DEV)
    for cap, want in ((r["fp"] - 1, hj.HJ_ERR_CAPACITY), (r["fp"], hj.HJ_OK)):
        sv = hj.Server(ws, mem_cap_bytes=cap, slots=1, max_batch_jobs=4)
        t = sv.submit(*r["t"], counts[0:1], r["p"], 0)  # declared footprint 0
        sv.drain()
        done = {tk: st for tk, st, _, _ in sv.poll()}
        assert done[t] == want, (cap, done)
        sv.close()
    assert int(counts[0].item()) == r["cap"]


def test_many_small_requests():
    n = 400
    r, s = gen.unique_uniform(30, 2048, 8192, 3000)
    rk, rr, sk, sr = (torch.from_numpy(a).to(DEV) for a in (r.key, r.rid, s.key, s.rid))
    want = oracle.join_count(r.key, r.rid, s.key)
    outs = torch.empty((n, 2, want), dtype=torch.int32, device=DEV)
    counts = torch.zeros(n, dtype=torch.int64, device=DEV)
    ws = torch.empty(256 << 20, dtype=torch.uint8, device=DEV)
    sv = hj.Server(ws, mem_cap_bytes=1 << 30, slots=2, max_batch_jobs=32)
    p = hj.params("phj", 0, (0, 0))
    for i in range(n):
        sv.submit(rk, rr, sk, sr, outs[i, 0], outs[i, 1], counts[i:i + 1], p, 1 << 20)
    sv.drain()
    done = sv.poll(1024)
    assert len(done) == n and all(x[1] == hj.HJ_OK for x in done)
    assert torch.all(counts == want)
    lat = np.array([x[2] for x in done])
    assert np.all(lat > 0)
    sv.close()
    ref = oracle.canonical(*oracle.join(r.key, r.rid, s.key, s.rid))
    for i in (0, n // 2, n - 1):
        assert np.array_equal(oracle.canonical(outs[i, 0].cpu().numpy(), outs[i, 1].cpu().numpy()), ref)


def test_drain_after_only_rejections():
    """drain() returns when the only requests were rejected at admission (nothing
    ever ran, so no finished batch wakes it)."""
    r, s = gen.unique_uniform(31, 2048, 4096, 3000)
    rk, rr, sk, sr = (torch.from_numpy(a).to(DEV) for a in (r.key, r.rid, s.key, s.rid))
    o = torch.empty((2, 4096), dtype=torch.int32, device=DEV)
    counts = torch.zeros(2, dtype=torch.int64, device=DEV)
    ws = torch.empty(64 << 20, dtype=torch.uint8, device=DEV)
    sv = hj.Server(ws, mem_cap_bytes=1 << 20, slots=2, max_batch_jobs=4)
    p = hj.params("phj", 0, (0, 0))
    t = [sv.submit(rk, rr, sk, sr, o[0], o[1], counts[i:i + 1], p, 2 << 20) for i in range(2)]
    sv.drain()
    done = {x[0]: x[1] for x in sv.poll()}
    assert done == {t[0]: hj.HJ_ERR_CAPACITY, t[1]: hj.HJ_ERR_CAPACITY}
    st = sv.stats()
    assert st["rejected"] == 2 and st["completed"] == 0 and st["bytes_in_use"] == 0
    sv.close()


def test_resident_tables_serve_probes():
    """Tables built once stay on the device and serve probe requests mixed with
    full joins; every probe equals the oracle's join of the table's R with its S."""
    r1, _ = gen.unique_uniform(32, 60000, 10, 1)
    r2, _ = gen.unique_uniform(33, 3000, 10, 1)
    tabs = [hj.Table(*(torch.from_numpy(a).to(DEV) for a in (r.key, r.rid)), p=p)
            for r, p in ((r1, hj.params("phj", 2, (4, 3), one_pass=True)), (r2, hj.params("shj")))]
    rels = [r1, r2]
    torch.cuda.synchronize()
    reqs = requests(34, 12, r_max=1 << 15)
    ws = torch.empty(1 << 29, dtype=torch.uint8, device=DEV)
    sv = hj.Server(ws, mem_cap_bytes=16 << 30, slots=4, max_batch_jobs=8)
    counts = torch.zeros(len(reqs) + 20, dtype=torch.int64, device=DEV)
    probes = []
    for i in range(20):
        k = i % 2
        _, s = gen.unique_uniform(100 + i, 10, 5000 + 997 * i, 2 * len(rels[k]))
        sk, sr = (torch.from_numpy(a).to(DEV) for a in (s.key, s.rid))
        o = torch.full((2, len(s)), -1, dtype=torch.int32, device=DEV)
        c = counts[len(reqs) + i: len(reqs) + i + 1]
        probes.append((k, s, o, c, sv.submit_probe(tabs[k], sk, sr, o[0], o[1], c, 1 << 20)))
        if i < len(reqs):
            r = reqs[i]
            sv.submit(*r["t"], counts[i:i + 1], r["p"], r["fp"])
    sv.drain()
    done = {t: st for t, st, _, _ in sv.poll()}
    assert all(st == hj.HJ_OK for st in done.values()) and len(done) == 20 + min(20, len(reqs))
    sv.close()
    for k, s, o, c, t in probes:
        n = int(c.item())
        w_r, w_s = oracle.join(rels[k].key, rels[k].rid, s.key, s.rid)
        assert n == len(w_r)
        assert np.array_equal(oracle.canonical(o[0, :n].cpu().numpy(), o[1, :n].cpu().numpy()),
                              oracle.canonical(w_r, w_s))
    got = counts[: len(reqs)].cpu().numpy()
    for i, r in enumerate(reqs):
        assert int(got[i]) == r["cap"]
