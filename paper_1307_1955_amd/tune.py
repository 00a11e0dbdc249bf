"""Planning support for per-join parameters: calibration and Monte-Carlo
validation of the cost model, and an autotuner on top of it.

The paper picks its co-processing ratios with a cost model (Section 4, Eq. 2-3:
a step's time is its computation plus its memory stalls plus its delay behind
the previous step) and validates the model Monte-Carlo style against
measurements over a thousand random settings, finding it within 15% in most
runs (Section 5.3).  Here the model (costmodel.py, compiled into the library
as csrc/costmodel.cpp) prices the launch sequence of a join, and HJ_AUTO runs
the candidate plan it rates fastest; batch planning without explicit
parameters does the same.  This module

* ``--collect``: times every kernel of a grid of joins on the device (the
  calibration data);
* ``--fit``: fits the model's constants to those times and writes
  tuning/mi355x_calib.json and the include the library compiles;
* ``--validate``: a thousand random settings (sizes over the batched
  workload's range, match rates, algorithm, passes, radix bits, tile, output
  mode), each timed on the device next to the library's prediction; writes the
  error distribution, the buckets where it misses 15%, and, for a few
  workloads, where the model's own choice falls among the random settings;
* the autotuner (default): per (|R|, |S|/|R|) bucket, the model ranks the
  candidates, the best few are timed and the fastest is stored in a table a
  batch may be planned with instead of the model.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
from dataclasses import dataclass

PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(PKG, "tuning", "mi355x_tuned.json")
MAX_RADIX_BITS = 20  # the library's limit on the radix bits of all passes


@dataclass(frozen=True)
class Candidate:
    algo: str            # "shj" | "phj" | "auto" (the library's HJ_AUTO choice: the cost model's)
    passes: int          # PHJ: 0 (direct), 1, 2
    bits: tuple = (0, 0)
    one_pass: bool = True
    tile: int = 0        # partition tile (0: the library's choice)

    def params(self):
        from . import hj
        if self.algo == "auto":
            return hj.params("auto", tile=self.tile, one_pass=self.one_pass)
        return hj.params(self.algo, self.passes, self.bits, tile=self.tile, one_pass=self.one_pass)

    def as_dict(self) -> dict:
        return {"algo": self.algo, "passes": self.passes, "bits": list(self.bits), "one_pass": self.one_pass,
                "tile": self.tile}

    @staticmethod
    def from_dict(d: dict) -> "Candidate":
        return Candidate(d["algo"], int(d["passes"]), tuple(d["bits"]), bool(d["one_pass"]), int(d.get("tile", 0)))


def _bits_for(n_r: int, target: int = 4096) -> int:
    b = 0
    while b < MAX_RADIX_BITS and (n_r >> b) > target:
        b += 1
    return b


def candidates(n_r: int, n_s: int) -> list[Candidate]:
    """The model's own pick (HJ_AUTO) and the plans around it."""
    out = [Candidate("auto", 0), Candidate("shj", 0), Candidate("shj", 0, one_pass=False)]
    if n_r <= 8192:
        out.append(Candidate("phj", 0))
    B = _bits_for(n_r)
    for b in sorted({max(1, B - 1), max(1, B), B + 1}):
        for tile in (4096, 8192):
            if b <= 13:
                out.append(Candidate("phj", 1, (b, 0), tile=tile))
            if 2 <= b <= MAX_RADIX_BITS:
                out.append(Candidate("phj", 2, ((b + 1) // 2, b // 2), tile=tile))
        if 2 <= b <= MAX_RADIX_BITS:
            out.append(Candidate("phj", 2, ((b + 1) // 2, b // 2), one_pass=False))
    return out


def model_ms(c: Candidate, n_r: int, n_s: int, m: float) -> float:
    """The library's cost-model time of candidate c (ms), inf if invalid."""
    from . import hj
    try:
        return hj.hj_model_seconds(c.params(), n_r, n_s, int(m)) * 1e3
    except hj.HJError:
        return math.inf


def bucket_key(n_r: int, n_s: int) -> tuple[int, int]:
    lr = int(round(math.log2(max(1, n_r))))
    ratio = max(1, n_s / max(1, n_r))
    rb = 0 if ratio < 2.5 else (1 if ratio < 8 else 2)
    return lr, rb


RATIO_OF_BUCKET = {0: 1, 1: 4, 2: 16}


def steady_join_ms(run, reps: int = 3, warm_ms: float = 2.0, span_ms: float = 1.0, cap: int = 200) -> float:
    """Mean device time (ms) of run() (one join enqueued on the current stream)
    at steady clocks: joins are run until at least warm_ms of device time has
    passed (the clocks ramp up under load), then at least `reps` joins covering
    at least span_ms are timed between two events."""
    import torch
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    done, spent, last = 0, 0.0, 0.0
    while done < cap and (done < 2 or spent < warm_ms):
        a.record()
        run()
        b.record()
        torch.cuda.synchronize()
        last = a.elapsed_time(b)
        spent += last
        done += 1
    k = max(reps, min(cap, int(math.ceil(span_ms / max(last, 1e-3)))))
    a.record()
    for _ in range(k):
        run()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / k


def measure(c: Candidate, n_r: int, n_s: int, domain: int, reps: int = 5, seed: int = 11, t=None) -> float:
    """Mean device time (s) of one hj_join with candidate c at steady clocks
    (steady_join_ms)."""
    import torch

    from . import hj
    from .gen import device as dgen
    if t is None:
        t = dgen.unique_uniform(seed, n_r, n_s, domain)
    p = c.params()
    ws = hj.workspace(p, n_r, n_s)
    out_r = torch.empty(max(1, n_s), dtype=torch.int32, device="cuda")
    out_s = torch.empty_like(out_r)
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    return steady_join_ms(lambda: hj.hj_join(p, *t, out_r, out_s, ws, d), reps) * 1e-3


def tune(log2_r=range(10, 23), ratios=(0, 1, 2), top: int = 4, match: float = 0.625, verbose=True) -> dict:
    """Times the model's best `top` candidates for every bucket; returns the table."""
    table = {"device": "MI355X (gfx950)", "method": "library cost model ranks, best few timed", "buckets": {}}
    for lr in log2_r:
        for rb in ratios:
            n_r = 1 << lr
            n_s = n_r * RATIO_OF_BUCKET[rb]
            dom = max(n_r, int(math.ceil(n_r / match)))
            m = n_s * n_r / dom
            cands = sorted(candidates(n_r, n_s), key=lambda c: model_ms(c, n_r, n_s, m))[:top]
            timed = [(measure(c, n_r, n_s, dom), c) for c in cands]
            timed.sort(key=lambda x: x[0])
            best_t, best = timed[0]
            table["buckets"]["%d:%d" % (lr, rb)] = {
                "n_r": n_r, "n_s": n_s, "best": best.as_dict(), "ms": round(best_t * 1e3, 4),
                "timed": [{"cand": c.as_dict(), "ms": round(t_ * 1e3, 4),
                           "model_ms": round(model_ms(c, n_r, n_s, m), 4)} for t_, c in timed],
            }
            if verbose:
                print("tune %2d:%d best %s %.4f ms" % (lr, rb, best.as_dict(), best_t * 1e3), file=sys.stderr,
                      flush=True)
    return table


def load_table(path: str = DEFAULT_TABLE) -> dict | None:
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def choose(n_r: int, n_s: int, table: dict | None = None) -> Candidate:
    """A job's candidate: the tuned table's bucket when a table is given (nearest
    |R| bucket), else the cost model's choice (HJ_AUTO)."""
    if table:
        lr, rb = bucket_key(n_r, n_s)
        lrs = sorted({int(k.split(":")[0]) for k in table["buckets"]})
        lr = min(lrs, key=lambda x: abs(x - lr))
        e = table["buckets"].get("%d:%d" % (lr, rb))
        if e:
            c = Candidate.from_dict(e["best"])
            if c.algo == "phj" and c.passes == 0 and n_r > 8192:
                c = Candidate("auto", 0)
            return c
    return Candidate("auto", 0)


def main():
    ap = argparse.ArgumentParser(description="calibrate, validate and tune the join planner on the GPU")
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--min-log2", type=int, default=10)
    ap.add_argument("--max-log2", type=int, default=22)
    ap.add_argument("--top", type=int, default=4)
    ap.add_argument("--collect", metavar="OUT", default=None,
                    help="time every kernel of the calibration grid and write the raw records to OUT")
    ap.add_argument("--quick", action="store_true", help="with --collect: every 7th setting only")
    ap.add_argument("--random", type=int, default=0, metavar="N",
                    help="with --collect: N random settings drawn like the validation's instead of the grid")
    ap.add_argument("--seed", type=int, default=7, help="with --collect --random: the draw's seed")
    ap.add_argument("--fit", metavar="RAW", nargs="+", default=None,
                    help="fit the cost model to the RAW files (from --collect); writes tuning/mi355x_calib.json "
                         "and the library's include")
    ap.add_argument("--validate", metavar="OUT", default=None,
                    help="Monte-Carlo validation of the library's model on random settings; writes OUT (JSON) "
                         "and OUT with .md")
    ap.add_argument("--runs", type=int, default=1000, help="with --validate: random settings")
    a = ap.parse_args()
    if a.collect:
        collect(a.collect, quick=a.quick, settings=calibration_random(a.random, a.seed) if a.random else None)
        return
    if a.fit:
        fit_calibration(a.fit)
        return
    if a.validate:
        validate(a.validate, a.runs)
        return
    table = tune(range(a.min_log2, a.max_log2 + 1), top=a.top)
    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1)
    print(a.out)


# ---------------------------------------------------------------------------
# Calibration data for the per-step cost model (Section 4: a step's time is its
# computation, its memory stalls and its delay behind the previous step; here
# every kernel launch is a step, timed with HIP events on the device).
# ---------------------------------------------------------------------------


def calibration_grid(quick: bool = False) -> list[dict]:
    """Join settings whose per-kernel times calibrate the model: PHJ with one and
    two radix passes over a range of fan-outs, tiles and both output modes, the
    direct LDS join, and SHJ, over |R| = 2^10..2^24, |S| = 1..16 x |R| and match
    rates of 25-100%."""
    g = []
    sizes = [1 << e for e in range(10, 25, 2)]
    for n_r in sizes:
        for ratio in (1, 4, 16):
            n_s = n_r * ratio
            if n_r + n_s > (1 << 26):
                continue
            for match in (0.25, 1.0):
                base = dict(n_r=n_r, n_s=n_s, match=match)
                for one in (True, False):
                    g.append(dict(base, algo="shj", passes=0, bits=(0, 0), tile=0, one_pass=one))
                if n_r <= 8192:
                    g.append(dict(base, algo="phj", passes=0, bits=(0, 0), tile=0, one_pass=True))
                B = _bits_for(n_r)
                for b in sorted({max(1, B - 2), max(1, B), min(13, B + 2)}):
                    for tile in (4096, 8192):
                        for one in (True, False):
                            g.append(dict(base, algo="phj", passes=1, bits=(b, 0), tile=tile, one_pass=one))
                if B >= 4:
                    for b1 in sorted({(B + 1) // 2, max(2, B // 2 - 1)}):
                        b2 = max(1, B - b1)
                        for tile in (4096, 8192):
                            g.append(dict(base, algo="phj", passes=2, bits=(b1, b2), tile=tile, one_pass=True))
                        g.append(dict(base, algo="phj", passes=2, bits=(b1, b2), tile=0, one_pass=False))
    return g[::7] if quick else g


def calibration_random(n: int, seed: int) -> list[dict]:
    """Join settings drawn the way the Monte-Carlo validation draws them (sizes,
    match rate and parameters at random), for calibrating on more than the
    regular grid; a different seed than the validation's keeps the two apart."""
    import numpy as np
    rng = np.random.default_rng(seed)
    g = []
    for _ in range(n):
        n_r = int(round(1024 * 4096 ** rng.random()))
        n_s = n_r * int(rng.integers(1, 17))
        match = float(rng.uniform(0.25, 1.0))
        c = random_setting(rng, n_r)
        bits = tuple(c.bits) if c.algo == "phj" and c.passes else (0, 0)
        g.append(dict(n_r=n_r, n_s=n_s, match=match, algo=c.algo, passes=c.passes, bits=bits,
                      tile=c.tile if c.algo == "phj" and c.passes else 0, one_pass=c.one_pass))
    return g


def collect(out_path: str, reps: int = 3, quick: bool = False, settings: list | None = None) -> None:
    """Times every kernel of every setting (the calibration grid unless given;
    reps joins each, HIP events per launch, after steady_join_ms has warmed the
    clocks and timed the whole join) and writes the raw records as JSON."""
    import torch

    from . import hj
    from .gen import device as dgen
    recs = []
    grid = settings if settings is not None else calibration_grid(quick)
    cache = {}
    for i, c in enumerate(grid):
        key = (c["n_r"], c["n_s"], c["match"])
        if key not in cache:
            cache.clear()
            torch.cuda.empty_cache()
            dom = max(c["n_r"], int(math.ceil(c["n_r"] / c["match"])))
            t = dgen.unique_uniform(11 + i, c["n_r"], c["n_s"], dom)
            out_r = torch.empty(max(1, c["n_s"]), dtype=torch.int32, device="cuda")
            out_s = torch.empty_like(out_r)
            cache[key] = (t, out_r, out_s, int((t[2] <= c["n_r"]).sum()))
        t, out_r, out_s, m = cache[key]
        p = hj.params(c["algo"], c["passes"], c["bits"], tile=c["tile"], one_pass=c["one_pass"])
        q = hj.hj_resolve_params(p, c["n_r"], c["n_s"])
        ws = hj.workspace(p, c["n_r"], c["n_s"])
        d = torch.zeros(1, dtype=torch.int64, device="cuda")
        join_ms = steady_join_ms(lambda: hj.hj_join(p, *t, out_r, out_s, ws, d), reps)
        launches = []
        for _ in range(reps):
            launches.append(hj.hj_join_timed(p, *t, out_r, out_s, ws, d))
        if int(d.item()) != m:
            raise AssertionError("calibration join %r gave %d pairs, expected %d" % (c, int(d.item()), m))
        names = [n for n, _ in launches[0]]
        ms = [sum(L[j][1] for L in launches) / reps for j in range(len(names))]
        recs.append({"cfg": {**c, "bits": list(c["bits"])}, "resolved": {
            "algo": q.algo, "passes": q.passes, "bits": [q.bits[0], q.bits[1]], "tile": q.tile,
            "lds_cap": q.lds_cap, "one_pass": bool(q.flags & hj.HJ_FLAG_ONE_PASS)},
            "pairs": m, "kernels": list(zip(names, ms)), "join_ms": join_ms})
        del ws
        if i % 25 == 0:
            print("collect %d/%d %s %.4f ms" % (i, len(grid), c, recs[-1]["join_ms"]), file=sys.stderr, flush=True)
    with open(out_path, "w") as f:
        json.dump({"device": torch.cuda.get_device_name(0), "reps": reps, "records": recs}, f)
    print(out_path)


def fit_calibration(raw_paths) -> None:
    """Fits the model to raw per-kernel times (one or more --collect files) and
    writes the calibration JSON and the C++ include (the library must be
    rebuilt afterwards)."""
    from . import costmodel
    if isinstance(raw_paths, str):
        raw_paths = [raw_paths]
    raw = {"records": []}
    for path in raw_paths:
        with open(path) as f:
            r = json.load(f)
        raw.setdefault("device", r.get("device"))
        raw["records"] += r["records"]
    params, report = costmodel.fit(raw)
    rec = {"device": raw.get("device", "MI355X"), "source": "tune.py --fit of %d joins (%d launches)" % (
        report["joins"], report["launches"]), "params": params, "fit": report}
    with open(costmodel.CALIB_JSON, "w") as f:
        json.dump(rec, f, indent=1)
    costmodel.write_inc(params)
    print(json.dumps(report, indent=1))
    print(costmodel.CALIB_JSON, costmodel.CALIB_INC)


def random_setting(rng, n_r: int) -> Candidate:
    """A random parameter setting for |R| = n_r: SHJ or PHJ (no partitioning when
    R fits one LDS table, one or two radix passes with 2^B partitions around
    |R| / 4096 and a random split), random tile and output mode."""
    one = bool(rng.integers(0, 2))
    r = rng.random()
    if r < 0.2:
        return Candidate("shj", 0, one_pass=one)
    if n_r <= 8192 and r < 0.35:
        return Candidate("phj", 0)
    B = max(1, min(MAX_RADIX_BITS, _bits_for(n_r) + int(rng.integers(-2, 3))))
    tile = int(rng.choice([4096, 8192]))
    if B < 2 or B > 13 or rng.random() < 0.5:
        if B > 13:
            b1 = int(rng.integers(max(1, B - 13), min(13, B - 1) + 1))
            return Candidate("phj", 2, (b1, B - b1), one, tile)
        return Candidate("phj", 1, (B, 0), one, tile)
    b1 = int(rng.integers(max(1, B - 13), min(13, B - 1) + 1))
    return Candidate("phj", 2, (b1, B - b1), one, tile)


def validate(out_path: str, runs: int = 1000, seed: int = 2024) -> dict:
    """Monte-Carlo validation (Section 5.3's method): `runs` random settings --
    |R| log-uniform in [1024, 4194304], |S| = |R| x U{1..16}, match rate
    U[0.25, 1], random parameters -- each timed on the device and predicted by
    the library's model; plus, for four workloads, 60 random settings each
    timed next to the model's own choice (HJ_AUTO)."""
    import numpy as np
    import torch

    from . import hj
    from .gen import device as dgen
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(runs):
        n_r = int(round(1024 * 4096 ** rng.random()))
        n_s = n_r * int(rng.integers(1, 17))
        match = float(rng.uniform(0.25, 1.0))
        dom = max(n_r, int(math.ceil(n_r / match)))
        c = random_setting(rng, n_r)
        t = dgen.unique_uniform(1000 + i, n_r, n_s, dom)
        pairs = int((t[2] <= n_r).sum())
        meas = measure(c, n_r, n_s, dom, reps=3, t=t)
        pred = hj.hj_model_seconds(c.params(), n_r, n_s, pairs)
        q = hj.hj_resolve_params(c.params(), n_r, n_s)
        rows.append({"n_r": n_r, "n_s": n_s, "pairs": pairs, "cand": c.as_dict(), "tile": q.tile,
                     "lds_cap": q.lds_cap, "measured_ms": meas * 1e3, "model_ms": pred * 1e3,
                     "err": pred / meas - 1.0})
        del t
        if i % 50 == 0:
            print("validate %d/%d %s err %+.3f" % (i, runs, c.as_dict(), rows[-1]["err"]), file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
    choice = []
    for lg, ratio in ((12, 8), (16, 4), (20, 4), (22, 2)):
        n_r = 1 << lg
        n_s = n_r * ratio
        dom = int(n_r / 0.625)
        t = dgen.unique_uniform(77 + lg, n_r, n_s, dom)
        pairs = int((t[2] <= n_r).sum())
        times = [measure(random_setting(rng, n_r), n_r, n_s, dom, reps=3, t=t) * 1e3 for _ in range(60)]
        auto = measure(Candidate("auto", 0), n_r, n_s, dom, reps=3, t=t) * 1e3
        q = hj.hj_resolve_params(hj.params("auto", one_pass=True), n_r, n_s)
        choice.append({"n_r": n_r, "n_s": n_s, "pairs": pairs, "auto_ms": auto, "auto_plan": repr(q),
                       "random_best_ms": min(times), "random_median_ms": float(np.median(times)),
                       "auto_rank_fraction": float(np.mean(np.array(times) < auto))})
        del t
    res = {"runs": rows, "model_choice": choice, "summary": summarize_validation(rows)}
    with open(out_path, "w") as f:
        json.dump(res, f)
    with open(os.path.splitext(out_path)[0] + ".md", "w") as f:
        f.write(validation_markdown(res))
    print(json.dumps(res["summary"], indent=1))
    return res


def _bucket_of(r: dict) -> str:
    c = r["cand"]
    kind = c["algo"] if c["algo"] == "shj" else ("direct" if c["passes"] == 0 else "phj%d" % c["passes"])
    return "%s, |R| 2^%d-2^%d" % (kind, 2 * (int(math.log2(r["n_r"])) // 2), 2 * (int(math.log2(r["n_r"])) // 2) + 1)


def summarize_validation(rows: list) -> dict:
    import numpy as np
    e = np.abs(np.array([r["err"] for r in rows]))
    s = {"runs": len(rows), "within_15pct": float(np.mean(e <= 0.15)),
         "abs_err_percentiles": {str(q): float(np.percentile(e, q)) for q in (10, 25, 50, 75, 90, 95, 99)},
         "signed_err_median": float(np.median([r["err"] for r in rows])), "buckets": {}}
    groups = {}
    for r in rows:
        groups.setdefault(_bucket_of(r), []).append(abs(r["err"]))
    for k in sorted(groups):
        v = np.array(groups[k])
        s["buckets"][k] = {"runs": len(v), "within_15pct": float(np.mean(v <= 0.15)), "median_abs_err": float(np.median(v))}
    s["buckets_missing_15pct"] = sorted(k for k, b in s["buckets"].items() if b["median_abs_err"] > 0.15)
    return s


def validation_markdown(res: dict) -> str:
    s = res["summary"]
    lines = ["# Cost model against measurement on MI355X (Monte Carlo, %d random settings)" % s["runs"], "",
             "Command: `python -m paper_1307_1955_amd.tune --validate <out>.json` (settings: |R| log-uniform in "
             "[1024, 4194304], |S| = |R| x U{1..16}, match rate U[0.25, 1], random algorithm, passes, radix bits, "
             "tile and output mode; each timed at steady clocks (at least 2 ms of warm-up joins, then at least 3 joins "
             "and 1 ms timed), predicted by "
             "`hj_model_seconds` with the true pair count).", "",
             "Within 15%% of the measured time: **%.1f%%** of the settings; median signed error %+.1f%%." % (
                 100 * s["within_15pct"], 100 * s["signed_err_median"]), "",
             "| abs error percentile | 10 | 25 | 50 | 75 | 90 | 95 | 99 |", "|---|---|---|---|---|---|---|---|",
             "| error | " + " | ".join("%.1f%%" % (100 * s["abs_err_percentiles"][q])
                                     for q in ("10", "25", "50", "75", "90", "95", "99")) + " |", "",
             "| bucket | runs | within 15% | median abs error |", "|---|---:|---:|---:|"]
    for k, b in s["buckets"].items():
        lines.append("| %s | %d | %.0f%% | %.1f%% |" % (k, b["runs"], 100 * b["within_15pct"], 100 * b["median_abs_err"]))
    lines += ["", "Buckets whose median error exceeds 15%%: %s." % (", ".join(s["buckets_missing_15pct"]) or "none"),
              "", "The model's own choice (HJ_AUTO) against 60 random settings of the same workload:", "",
              "| |R| | |S| | HJ_AUTO plan | HJ_AUTO ms | best random ms | median random ms | random settings faster |",
              "|---:|---:|---|---:|---:|---:|---:|"]
    for c in res["model_choice"]:
        lines.append("| %d | %d | `%s` | %.4f | %.4f | %.4f | %.0f%% |" % (
            c["n_r"], c["n_s"], c["auto_plan"], c["auto_ms"], c["random_best_ms"], c["random_median_ms"],
            100 * c["auto_rank_fraction"]))
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    main()
