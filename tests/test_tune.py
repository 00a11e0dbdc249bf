"""The autotuner's host logic (no GPU): its mirror of the library's HJ_AUTO rule
agrees with what the library resolves, and the cost model prices every
candidate."""
import math

import pytest

from paper_1307_1955_amd import tune


@pytest.fixture(scope="module")
def hj():
    import paper_1307_1955_amd.hj as m
    m.load()
    return m


SIZES = [1, 4416, 4417, 9000, 65536, 100000, 1 << 20, (1 << 22) - 1, 1 << 22, (1 << 22) + 4096, 1 << 24, 3 << 24,
         1 << 30, (1 << 31) - 1, 80_000_000, 300_000_000, 1_200_000_000]


@pytest.mark.parametrize("n_r", SIZES)
def test_auto_candidate_matches_library(hj, n_r):
    c = tune.auto_candidate(n_r)
    for n_s in (1000, 1 << 24):
        q = hj.hj_resolve_params(hj.params("auto", one_pass=True), n_r, n_s)
        assert (q.passes, tuple(q.bits)) == (c.passes, tuple(c.bits))
        if c.passes:
            # the tile the cost model assumes for HJ_AUTO is the library's
            big = n_r + n_s >= 1 << 25 or (n_r + n_s >= 1 << 24 and c.passes == 1 and c.bits[0] >= 8)
            assert q.tile == (8192 if big else 4096)


@pytest.mark.parametrize("n_r,n_s", [(1 << 12, 1 << 16), (1 << 16, 1 << 20), (1 << 20, 1 << 24), (1 << 22, 1 << 22)])
def test_model_prices_every_candidate(n_r, n_s):
    cands = tune.candidates(n_r, n_s)
    assert any(c.algo == "auto" for c in cands)
    for c in cands:
        t = tune.predict(c, n_r, n_s, 0.5 * n_s)
        assert math.isfinite(t) and t > 0
    # HJ_AUTO is priced as the concrete candidate it resolves to, with the library's tile
    x = tune.auto_candidate(n_r)
    n = n_r + n_s
    tile = 8192 if (n >= 1 << 25 or (n >= 1 << 24 and x.passes == 1 and x.bits[0] >= 8)) else 4096
    want = tune.predict(tune.Candidate(x.algo, x.passes, x.bits, True, tile), n_r, n_s, 0.5 * n_s)
    assert tune.predict(tune.Candidate("auto", 0), n_r, n_s, 0.5 * n_s) == want


def test_table_round_trip():
    c = tune.Candidate("auto", 0)
    assert tune.Candidate.from_dict(c.as_dict()) == c
    d = tune.Candidate("phj", 2, (5, 4), False, 8192)
    assert tune.Candidate.from_dict(d.as_dict()) == d
