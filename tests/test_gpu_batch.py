"""GPU parity of batched joins: every job of a batch against the oracle, and
the same job alone; graph replays checked one by one."""
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


def make_jobs(seed, sizes, dup=False):
    """Host relations and device tensors for jobs of the given (|R|, |S|, S key domain)."""
    rng = np.random.default_rng(seed)
    host, dev = [], []
    for i, (nr, ns, dom) in enumerate(sizes):
        r, s = gen.unique_uniform(seed * 1000 + i, nr, ns, dom)
        rk, sk = r.key.copy(), s.key.copy()
        if dup and nr:
            rk[rng.integers(0, nr, size=max(1, nr // 20))] = rk[0]
        host.append((rk, r.rid, sk, s.rid))
        cap = max(1, int(oracle.join_count(rk, r.rid, sk)))
        t = [torch.from_numpy(a).to(DEV) for a in (rk, r.rid, sk, s.rid)]
        t += [torch.full((cap,), -1, dtype=torch.int32, device=DEV) for _ in range(2)]
        dev.append(t)
    return host, dev


SIZES = [
    (1000, 3000, 1500), (4096, 4096, 8192), (4416, 9000, 5000), (0, 100, 10), (100, 0, 10),
    (5000, 20000, 6000), (70000, 140000, 100000), (300000, 300000, 600000), (2000, 50000, 2000),
    (1, 1, 1), (8192, 8192, 8192), (17, 300000, 40), (1 << 20, 1 << 20, 1 << 21),
]


def check_jobs(host, dev, counts):
    for j, ((rk, rr, sk, sr), t) in enumerate(zip(host, dev)):
        want_r, want_s = oracle.join(rk, rr, sk, sr)
        c = int(counts[j])
        assert c == len(want_r), (j, c, len(want_r))
        got = oracle.canonical(t[4][:c].cpu().numpy(), t[5][:c].cpu().numpy())
        assert np.array_equal(got, oracle.canonical(want_r, want_s)), j


@pytest.mark.parametrize("graph", [True, False])
def test_batch_default_rule(graph):
    host, dev = make_jobs(1, SIZES, dup=True)
    d_counts = torch.zeros(len(dev), dtype=torch.int64, device=DEV)
    plan = hj.BatchPlan(dev, d_counts, graph=graph)
    assert plan.direct_jobs >= 5
    ws = plan.workspace()
    plan.run(ws)
    torch.cuda.synchronize()
    check_jobs(host, dev, d_counts.cpu().numpy())
    plan.close()


def test_batch_explicit_params_and_same_alone():
    sizes = SIZES[:9]
    host, dev = make_jobs(2, sizes)
    params = []
    for j, (nr, ns, dom) in enumerate(sizes):
        kind = j % 5
        if kind == 0 and nr <= 8192:
            params.append(hj.params("phj", 0, (0, 0)))
        elif kind == 1:
            params.append(hj.params("shj"))
        elif kind == 2:
            params.append(hj.params("phj", 1, (3,)))
        elif kind == 3:
            params.append(hj.params("phj", 2, (2, 2), one_pass=True))
        else:
            params.append(hj.params("shj", one_pass=True))
    d_counts = torch.zeros(len(dev), dtype=torch.int64, device=DEV)
    plan = hj.BatchPlan(dev, d_counts, params=params)
    plan.run(plan.workspace())
    torch.cuda.synchronize()
    check_jobs(host, dev, d_counts.cpu().numpy())
    # each job alone through hj_join gives the same multiset
    for j, t in enumerate(dev):
        o_r, o_s, cnt = hj.join(*t[:4], p=params[j])
        c = int(d_counts[j].item())
        assert cnt == c
        assert np.array_equal(oracle.canonical(o_r.cpu().numpy(), o_s.cpu().numpy()),
                              oracle.canonical(t[4][:c].cpu().numpy(), t[5][:c].cpu().numpy()))
    plan.close()


def test_graph_replays_each_checked():
    host, dev = make_jobs(3, SIZES[:8])
    d_counts = torch.zeros(len(dev), dtype=torch.int64, device=DEV)
    plan = hj.BatchPlan(dev, d_counts)
    ws = plan.workspace()
    assert plan.graph_nodes == 0  # nothing captured before the first run
    for rep in range(3):
        for t in dev:
            t[4].fill_(-1)
            t[5].fill_(-1)
        d_counts.fill_(-5)
        torch.cuda.synchronize()
        plan.run(ws)
        torch.cuda.synchronize()
        check_jobs(host, dev, d_counts.cpu().numpy())
        assert plan.graph_nodes >= len(dev)  # at least one kernel per job
        # unrelated eager work between replays
        x = torch.arange(1 << 20, device=DEV)
        assert int(x.sum().item()) == (1 << 20) * ((1 << 20) - 1) // 2
    plan.close()


def test_batch_capacity_per_job():
    host, dev = make_jobs(4, [(3000, 9000, 4000), (70000, 70000, 80000)])
    want = [oracle.join_count(h[0], h[1], h[2]) for h in host]
    short = []
    for t, w in zip(dev, want):
        o_r = torch.full((w,), -7, dtype=torch.int32, device=DEV)
        o_s = torch.full((w,), -7, dtype=torch.int32, device=DEV)
        short.append(t[:4] + [o_r[: w // 2], o_s[: w // 2], o_r, o_s])
    d_counts = torch.zeros(2, dtype=torch.int64, device=DEV)
    plan = hj.BatchPlan([s[:6] for s in short], d_counts)
    plan.run(plan.workspace())
    torch.cuda.synchronize()
    assert d_counts.cpu().tolist() == want
    for s, w in zip(short, want):
        assert torch.all(s[6][w // 2:] == -7) and torch.all(s[7][w // 2:] == -7)
    plan.close()


def test_batch_of_generated_jobs_device():
    """Jobs drawn like the batched workload (log-uniform |R|, |S| = k|R|), small scale."""
    specs = gen.batch_specs(7, 64, r_min=1024, r_max=1 << 16, max_factor=16)
    dev, host_specs = [], []
    for sp in specs:
        rk, rr, sk, sr = dgen.job_relations(sp)
        cap = sp.n_s
        dev.append([rk, rr, sk, sr, torch.empty(cap, dtype=torch.int32, device=DEV),
                    torch.empty(cap, dtype=torch.int32, device=DEV)])
        host_specs.append(sp)
    d_counts = torch.zeros(len(dev), dtype=torch.int64, device=DEV)
    plan = hj.BatchPlan(dev, d_counts)
    plan.run(plan.workspace())
    torch.cuda.synchronize()
    counts = d_counts.cpu().numpy()
    for j, sp in enumerate(host_specs):
        r, s = gen.job_relations(sp)
        c = int(counts[j])
        assert c == int(np.sum(s.key <= sp.n_r))  # closed form: R keys are 1..|R|
        m = oracle.match_of(dev[j][4][:c].cpu().numpy(), dev[j][5][:c].cpu().numpy(), sp.n_s)
        inv = np.empty(sp.n_r + 1, dtype=np.int64)
        inv[r.key] = np.arange(sp.n_r)
        expect = np.where(s.key <= sp.n_r, inv[np.minimum(s.key, sp.n_r)], -1)
        assert np.array_equal(m, expect), j
    plan.close()
