"""The planner's host logic (no GPU): candidate sets, the table round trip, the
model's fit on synthetic data, and the validation summary."""
import math

import numpy as np
import pytest

from paper_1307_1955_amd import costmodel, tune


@pytest.fixture(scope="module")
def hj():
    import paper_1307_1955_amd.hj as m
    m.load()
    return m


@pytest.mark.parametrize("n_r,n_s", [(1 << 10, 1 << 12), (1 << 12, 1 << 16), (1 << 16, 1 << 20), (1 << 20, 1 << 24),
                                     (1 << 22, 1 << 22)])
def test_model_prices_every_candidate(hj, n_r, n_s):
    cands = tune.candidates(n_r, n_s)
    assert cands[0] == tune.Candidate("auto", 0)
    ts = [tune.model_ms(c, n_r, n_s, n_s) for c in cands]  # HJ_AUTO plans for |S| pairs
    assert all(math.isfinite(t) and t > 0 for t in ts)
    # HJ_AUTO keeps the output mode and is the model's minimum over a superset of
    # these plans at the library's tile size rule, so no such candidate with the
    # same (one-pass) output beats it
    def rule_tile(c):
        if c.algo == "shj" or c.passes == 0:
            return c.tile
        p = c.params()
        p.tile = 0
        return hj.hj_resolve_params(p, n_r, n_s).tile
    same = [t for c, t in zip(cands[1:], ts[1:]) if c.one_pass and (c.tile == 0 or c.tile == rule_tile(c))]
    assert ts[0] <= min(same) * (1 + 1e-12)


def test_random_settings_are_valid(hj):
    rng = np.random.default_rng(3)
    for _ in range(400):
        n_r = int(round(1024 * 4096 ** rng.random()))
        c = tune.random_setting(rng, n_r)
        q = hj.hj_resolve_params(c.params(), n_r, n_r * 4)
        assert q.algo in (hj.HJ_SHJ, hj.HJ_PHJ)


def test_table_round_trip_and_choose():
    c = tune.Candidate("auto", 0)
    assert tune.Candidate.from_dict(c.as_dict()) == c
    d = tune.Candidate("phj", 2, (5, 4), False, 8192)
    assert tune.Candidate.from_dict(d.as_dict()) == d
    assert tune.choose(1 << 20, 1 << 22, None) == c
    table = {"buckets": {"20:1": {"best": d.as_dict()}}}
    assert tune.choose(1 << 20, 1 << 22, table) == d


def test_fit_recovers_known_constants():
    """The fit recovers constants from kernel times the model itself generates
    (the fitting machinery, independent of any device)."""
    truth = dict(costmodel.START)
    truth.update(bw_scatter=4.8e12, run_half=11.0, l_join0=6e-6, t_ins=1.2e-10, gamma_ins=-0.15, d_kernel=2.5e-6,
                 l_ovf_round=5e-6, d_gap=-1.5e-6)
    recs = []
    for n_r, n_s in [(1 << 12, 1 << 14), (1 << 16, 1 << 18), (1 << 20, 1 << 20), (1 << 22, 1 << 24), (1 << 24, 1 << 24)]:
        for plan in [{"algo": "shj", "passes": 0, "bits": (0, 0), "tile": 4096, "lds_cap": 0, "one_pass": o}
                     for o in (True, False)] + \
                    [{"algo": "phj", "passes": 1, "bits": (b, 0), "tile": t, "lds_cap": 4416, "one_pass": o}
                     for b in (4, 8, 12) for t in (4096, 8192) for o in (True, False)] + \
                    [{"algo": "phj", "passes": 2, "bits": (6, 6), "tile": 8192, "lds_cap": 4416, "one_pass": True}]:
            ls = costmodel.launches(plan, n_r, n_s, n_s // 2)
            ks = [(k, costmodel.kernel_seconds(k, f, truth) * 1e3) for k, f in ls]
            recs.append({"cfg": {"n_r": n_r, "n_s": n_s}, "resolved": {
                "algo": 0 if plan["algo"] == "shj" else 1, "passes": plan["passes"], "bits": list(plan["bits"]),
                "tile": plan["tile"], "lds_cap": plan["lds_cap"], "one_pass": plan["one_pass"]},
                "pairs": n_s // 2, "kernels": ks,
                "join_ms": costmodel.join_seconds(plan, n_r, n_s, n_s // 2, truth) * 1e3})
    params, report = costmodel.fit({"records": recs})
    assert report["join_abs_rel_err_p90"] < 0.02, report
    assert params["bw_scatter"] == pytest.approx(truth["bw_scatter"], rel=0.05)
    assert params["d_gap"] == pytest.approx(truth["d_gap"], rel=0.05)
    assert params["gamma_ins"] == pytest.approx(truth["gamma_ins"], abs=0.02)


def test_validation_summary_names_failing_buckets():
    rows = [{"n_r": 1 << 12, "n_s": 1 << 14, "cand": {"algo": "shj", "passes": 0}, "err": 0.05}] * 10 + \
           [{"n_r": 1 << 20, "n_s": 1 << 22, "cand": {"algo": "phj", "passes": 2}, "err": -0.4}] * 10
    s = tune.summarize_validation(rows)
    assert s["within_15pct"] == pytest.approx(0.5)
    assert s["buckets_missing_15pct"] == ["phj2, |R| 2^20-2^21"]
    md = tune.validation_markdown({"summary": s, "model_choice": []})
    assert "phj2, |R| 2^20-2^21" in md
