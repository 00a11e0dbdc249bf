"""GPU tests of the failure paths, forced from the host so every kernel still
ends normally (HJ_DEBUG_FAIL_PHASE, read by the library at every call):

* scan_stall: the first tile of every histogram and count scan (chained,
  decoupled look-back) withholds its status and the waits give up after 64 polls.  The call's error
  word must report it: hj_join_sync and hj_workspace_status return
  HJ_ERR_DEVICE, a batch reports it through its workspace, a server marks the
  requests of that batch HJ_ERR_DEVICE and keeps serving.  The next call on the
  same workspace, without the knob, is correct and clean again.
* launch:<phase>: a launch reports a failure; the call returns HJ_ERR_DEVICE,
  and a server stops admitting, fails its requests and releases their
  footprints.
"""
import os
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

DEV = torch.device("cuda:0")
KNOB = "HJ_DEBUG_FAIL_PHASE"


class knob:
    def __init__(self, value):
        self.value = value

    def __enter__(self):
        os.environ[KNOB] = self.value

    def __exit__(self, *exc):
        os.environ.pop(KNOB, None)


def relations(seed, n_r, n_s):
    r, s = gen.unique_uniform(seed, n_r, n_s, 2 * n_r)
    t = [torch.from_numpy(a).to(DEV) for a in (r.key, r.rid, s.key, s.rid)]
    return r, s, t


# every case has a chained scan over more than one tile (or a plan over several workgroups)
STALL_CASES = [
    ("phj2_6_6", dict(algo="phj", passes=2, bits=(6, 6))),
    ("phj2_6_6_1pass", dict(algo="phj", passes=2, bits=(6, 6), one_pass=True)),
    ("phj1_10", dict(algo="phj", passes=1, bits=(10,))),
    ("shj", dict(algo="shj")),
]


@pytest.mark.parametrize("name,kw", STALL_CASES, ids=[c[0] for c in STALL_CASES])
def test_scan_give_up_is_reported(name, kw):
    p = hj.params(**kw)
    r, s, t = relations(41, 1 << 18, 1 << 21)
    ws = hj.workspace(p, len(r), len(s))
    out_r = torch.empty(len(s), dtype=torch.int32, device=DEV)
    out_s = torch.empty(len(s), dtype=torch.int32, device=DEV)
    d = torch.zeros(1, dtype=torch.int64, device=DEV)
    with knob("scan_stall"):
        with pytest.raises(hj.HJError) as e:
            hj.hj_join_sync(p, *t, out_r, out_s, ws, d)
        assert e.value.status == hj.HJ_ERR_DEVICE
        assert "gave up" in e.value.message
        # the asynchronous form: the error word of its workspace
        hj.hj_join(p, *t, out_r, out_s, ws, d)
        with pytest.raises(hj.HJError) as e:
            hj.hj_workspace_status(ws)
        assert e.value.status == hj.HJ_ERR_DEVICE
    # the same workspace without the knob: cleared by the call, result correct
    cnt = hj.hj_join_sync(p, *t, out_r, out_s, ws, d)
    hj.hj_workspace_status(ws)
    want = oracle.canonical(*oracle.join(r.key, r.rid, s.key, s.rid))
    assert cnt == len(want)
    assert np.array_equal(oracle.canonical(out_r[:cnt].cpu().numpy(), out_s[:cnt].cpu().numpy()), want)


def test_scan_give_up_build_probe():
    p = hj.params("phj", 2, (6, 6))
    r, s, t = relations(42, 1 << 18, 1 << 20)
    with knob("scan_stall"):
        tab = hj.Table(t[0], t[1], p)
        with pytest.raises(hj.HJError):
            hj.hj_workspace_status(tab.ws)
    tab = hj.Table(t[0], t[1], p)
    hj.hj_workspace_status(tab.ws)
    o_r, o_s, cnt = tab.probe(t[2], t[3])
    want = oracle.canonical(*oracle.join(r.key, r.rid, s.key, s.rid))
    assert np.array_equal(oracle.canonical(o_r.cpu().numpy(), o_s.cpu().numpy()), want)


def test_scan_give_up_in_batch():
    """Lanes of a batch report into the batch's error word (run without a graph:
    a captured graph keeps the launch arguments of its capture)."""
    jobs, keep = [], []
    for i, (nr, ns) in enumerate([(1 << 16, 1 << 18), (1 << 17, 1 << 17), (3000, 9000)]):
        r, s, t = relations(50 + i, nr, ns)
        o_r = torch.empty(ns, dtype=torch.int32, device=DEV)
        o_s = torch.empty(ns, dtype=torch.int32, device=DEV)
        jobs.append([*t, o_r, o_s])
        keep.append((r, s))
    counts = torch.zeros(len(jobs), dtype=torch.int64, device=DEV)
    params = [hj.params("phj", 2, (6, 6), one_pass=True), hj.params("shj"), hj.params("auto", one_pass=True)]
    plan = hj.BatchPlan(jobs, counts, params=params, graph=False)
    ws = plan.workspace()
    with knob("scan_stall"):
        plan.run(ws)
        with pytest.raises(hj.HJError) as e:
            hj.hj_workspace_status(ws)
        assert e.value.status == hj.HJ_ERR_DEVICE
    plan.run(ws)
    hj.hj_workspace_status(ws)
    for j, (r, s) in enumerate(keep):
        c = int(counts[j].item())
        want = oracle.canonical(*oracle.join(r.key, r.rid, s.key, s.rid))
        assert c == len(want)
        got = oracle.canonical(jobs[j][4][:c].cpu().numpy(), jobs[j][5][:c].cpu().numpy())
        assert np.array_equal(got, want)
    plan.close()


def test_scan_give_up_in_server():
    """A server marks the requests of a batch whose error word is set HJ_ERR_DEVICE
    and keeps serving: later requests (without the knob) are correct."""
    r, s, t = relations(43, 1 << 17, 1 << 18)
    p = hj.params("phj", 2, (6, 6))
    fp = 16 * (len(r) + len(s)) + hj.hj_workspace_bytes(p, len(r), len(s))
    ws = torch.empty(1 << 28, dtype=torch.uint8, device=DEV)
    sv = hj.Server(ws, mem_cap_bytes=1 << 34, slots=2, max_batch_jobs=4)
    outs = [(torch.empty(len(s), dtype=torch.int32, device=DEV), torch.empty(len(s), dtype=torch.int32, device=DEV),
             torch.zeros(1, dtype=torch.int64, device=DEV)) for _ in range(2)]
    with knob("scan_stall"):
        bad = sv.submit(*t, *outs[0], p, fp)
        sv.drain()
        done = {tk: st for tk, st, *_ in sv.poll()}
    assert done[bad] == hj.HJ_ERR_DEVICE
    good = sv.submit(*t, *outs[1], p, fp)
    sv.drain()
    done = {tk: st for tk, st, *_ in sv.poll()}
    assert done[good] == hj.HJ_OK
    c = int(outs[1][2].item())
    want = oracle.canonical(*oracle.join(r.key, r.rid, s.key, s.rid))
    assert np.array_equal(oracle.canonical(outs[1][0][:c].cpu().numpy(), outs[1][1][:c].cpu().numpy()), want)
    assert sv.stats()["bytes_in_use"] == 0
    sv.close()


@pytest.mark.parametrize("phase,kw", [("part_scatter", dict(algo="phj", passes=2, bits=(6, 6))),
                                      ("shj_build", dict(algo="shj")),
                                      ("direct_join", dict(algo="phj", passes=0))])
def test_injected_launch_failure(phase, kw):
    p = hj.params(**kw)
    r, s, t = relations(44, 4000, 50000)
    ws = hj.workspace(p, len(r), len(s))
    out_r = torch.empty(len(s), dtype=torch.int32, device=DEV)
    out_s = torch.empty(len(s), dtype=torch.int32, device=DEV)
    d = torch.zeros(1, dtype=torch.int64, device=DEV)
    with knob("launch:" + phase):
        with pytest.raises(hj.HJError) as e:
            hj.hj_join(p, *t, out_r, out_s, ws, d)
        assert e.value.status == hj.HJ_ERR_DEVICE
    torch.cuda.synchronize()
    cnt = hj.hj_join_sync(p, *t, out_r, out_s, ws, d)
    assert cnt == oracle.join_count(r.key, r.rid, s.key)


def test_injected_launch_failure_server_releases_footprint():
    """A failed launch stops the server: the request fails, its footprint is
    released, drain returns and later submissions are refused."""
    r, s, t = relations(45, 1 << 16, 1 << 17)
    p = hj.params("phj", 2, (6, 6))
    ws = torch.empty(1 << 28, dtype=torch.uint8, device=DEV)
    sv = hj.Server(ws, mem_cap_bytes=1 << 34, slots=2, max_batch_jobs=4)
    o = (torch.empty(len(s), dtype=torch.int32, device=DEV), torch.empty(len(s), dtype=torch.int32, device=DEV),
         torch.zeros(1, dtype=torch.int64, device=DEV))
    with knob("launch:part_scatter"):
        tk = sv.submit(*t, *o, p, 12345678)
        with pytest.raises(hj.HJError):
            sv.drain()
        deadline = time.time() + 30
        while time.time() < deadline and sv.stats()["bytes_in_use"] != 0:
            time.sleep(0.01)
    torch.cuda.synchronize()
    assert sv.stats()["bytes_in_use"] == 0
    with pytest.raises(hj.HJError):
        sv.submit(*t, *o, p, 1)
    sv.close()
    assert tk >= 1
