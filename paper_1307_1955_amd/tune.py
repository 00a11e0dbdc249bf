"""Autotuner for per-job join parameters, seeded by a cost model.

The paper picks its co-processing ratios by evaluating a cost model over a
grid of candidates and keeping the best (Section 3.2, the delta-grid search;
the model is Section 4, Eq. 2-3: a step's time is its computation plus its
memory stalls).  Here the grid is over the join's own knobs -- SHJ or PHJ,
radix passes and bits, direct (unpartitioned) LDS join, one- or two-pass
output -- for buckets of (|R|, |S|/|R|).  The model ranks the candidates of a
bucket; the best few are then timed on the device and the fastest is stored
in a JSON table that batch planning looks up.

Model (per candidate): time = sum over phases of bytes / bandwidth(access
pattern) + launches * launch cost + work items * per-item cost, with the
bandwidths and costs calibrated on MI355X measurements of this library.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
from dataclasses import dataclass

PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(PKG, "tuning", "mi355x.json")

# Calibration on MI355X (rocprofv3 kernel times, 16M x 16M PHJ, 6+6 bits):
# histogram read 4 B/tuple in 31 us per pass; scatter 16 B/tuple in 110 us per
# pass; one-pass LDS join write (8 B/tuple + 8 B/pair) 95 us for 4096 work
# items of ~17 us each; SHJ build 16M tuples in 0.78 ms into a 256 MB table,
# probe 0.35 ms per pass.
CALIB = {
    "bw_hist": 4.3e12,          # B/s, streaming key read
    "bw_scatter": 4.9e12,       # B/s, read 8 + write 8 per tuple
    "bw_join": 3.5e12,          # B/s, LDS-table join passes
    "item_lat": 17e-6,          # s, one join work item start to finish
    "launch": 4e-6,             # s, per kernel launch
    "shj_build_hbm": 47e-9,     # s per R tuple, table beyond the caches
    "shj_build_cache": 4e-9,    # s per R tuple, table resident in L2 / MALL
    "shj_probe_hbm": 21e-9,     # s per S tuple per probe pass, table beyond the caches
    "shj_probe_cache": 1.5e-9,  # s per S tuple per probe pass, cached table
    "cache_bytes": 128 << 20,   # share of the 256 MB MALL a table can count on
    "cus": 256,
    "join_blocks_per_cu": 3,
}


@dataclass(frozen=True)
class Candidate:
    algo: str            # "shj" | "phj" | "auto" (the library's HJ_AUTO choice for the job's own sizes)
    passes: int          # PHJ: 0 (direct), 1, 2
    bits: tuple = (0, 0)
    one_pass: bool = True
    tile: int = 0        # partition tile (0: 4096, the tile the stored table was measured with)

    def params(self):
        from . import hj
        if self.algo == "auto":  # parameters and tile as the library chooses them
            return hj.params("auto", tile=self.tile, one_pass=self.one_pass)
        return hj.params(self.algo, self.passes, self.bits, tile=self.tile or 4096, one_pass=self.one_pass)

    def as_dict(self) -> dict:
        return {"algo": self.algo, "passes": self.passes, "bits": list(self.bits), "one_pass": self.one_pass,
                "tile": self.tile}

    @staticmethod
    def from_dict(d: dict) -> "Candidate":
        return Candidate(d["algo"], int(d["passes"]), tuple(d["bits"]), bool(d["one_pass"]), int(d.get("tile", 0)))


MAX_RADIX_BITS = 20  # the library's limit on the radix bits of all passes


def _bits_for(n_r: int, target: int = 4096) -> int:
    b = 0
    while b < MAX_RADIX_BITS and (n_r >> b) > target:
        b += 1
    return b


# HJ_AUTO's rule (the library's auto_params), for the cost model: no
# partitioning up to AUTO_DIRECT_MAX R tuples, else ~4096 R tuples per
# partition, one pass up to AUTO_ONE_PASS_MAX_BITS radix bits.
AUTO_DIRECT_MAX = 4416
AUTO_ONE_PASS_MAX_BITS = 10
AUTO_WIDE_FROM_BITS = 16  # above this, partitions of up to 5120 R tuples


def auto_candidate(n_r: int) -> Candidate:
    """The concrete candidate HJ_AUTO picks for |R| = n_r (tile left to the library)."""
    if n_r <= AUTO_DIRECT_MAX:
        return Candidate("phj", 0)
    b = _bits_for(n_r)
    if b > AUTO_WIDE_FROM_BITS:
        b = _bits_for(n_r, 5120)
    if b <= AUTO_ONE_PASS_MAX_BITS:
        return Candidate("phj", 1, (b, 0))
    return Candidate("phj", 2, ((b + 1) // 2, b // 2))


def candidates(n_r: int, n_s: int) -> list[Candidate]:
    out = [Candidate("shj", 0), Candidate("shj", 0, one_pass=False), Candidate("auto", 0)]
    if n_r <= 8192:
        out.append(Candidate("phj", 0))
    B = _bits_for(n_r)
    for b in {max(1, B - 1), max(1, B), B + 1}:
        if b <= AUTO_ONE_PASS_MAX_BITS:
            out.append(Candidate("phj", 1, (b, 0)))
        if 2 <= b <= 16:
            out.append(Candidate("phj", 2, ((b + 1) // 2, b // 2)))
            out.append(Candidate("phj", 2, ((b + 1) // 2, b // 2), one_pass=False))
    return out


def predict(c: Candidate, n_r: int, n_s: int, m: float, cal: dict = CALIB) -> float:
    """Cost-model time (s) of candidate c on |R| = n_r, |S| = n_s with m pairs."""
    if c.algo == "auto":
        a = auto_candidate(n_r)
        tile = 8192 if (n_r + n_s >= 1 << 25 or (n_r + n_s >= 1 << 24 and a.passes == 1 and a.bits[0] >= 8)) \
            else 4096
        return predict(Candidate(a.algo, a.passes, a.bits, c.one_pass, tile), n_r, n_s, m, cal)
    n = n_r + n_s
    conc = cal["cus"] * cal["join_blocks_per_cu"]
    if c.algo == "shj":
        table = 8 * (1 << max(1, math.ceil(math.log2(max(2, 2 * n_r)))))
        cached = table <= cal["cache_bytes"]
        build = n_r * (cal["shj_build_cache"] if cached else cal["shj_build_hbm"])
        probes = 1 if c.one_pass else 2
        probe = probes * n_s * (cal["shj_probe_cache"] if cached else cal["shj_probe_hbm"])
        out = 8 * m / cal["bw_join"]
        launches = 3 if c.one_pass else 7
        return build + probe + out + launches * cal["launch"]
    if c.passes == 0:
        items = math.ceil(n_s / 4096)
        waves = math.ceil(items / conc)
        return waves * cal["item_lat"] + (8 * n + 8 * m) / cal["bw_join"] + 2 * cal["launch"]
    t = 0.0
    tile = c.tile or 4096
    for b in c.bits[: c.passes]:
        # scatter runs shorter than ~64 tuples waste write bandwidth
        runs = tile / (1 << b)
        eff = min(1.0, runs / 64.0)
        t += 4 * n / cal["bw_hist"] + 16 * n / (cal["bw_scatter"] * max(eff, 0.25)) + 3 * cal["launch"]
    P = 1 << sum(c.bits[: c.passes])
    items = P + math.ceil(n_s / 4096)
    waves = math.ceil(items / conc)
    join_bytes = (8 * n + 8 * m) + (0 if c.one_pass else 4 * n)
    t += max(waves * cal["item_lat"], join_bytes / cal["bw_join"]) * (1 if c.one_pass else 1.6)
    t += (4 if c.one_pass else 6) * cal["launch"]
    r_part = n_r / P
    if r_part > 8192:  # partitions beyond the LDS budget take the HBM-table path
        t += n * cal["shj_probe_hbm"]
    return t


def bucket_key(n_r: int, n_s: int) -> tuple[int, int]:
    lr = int(round(math.log2(max(1, n_r))))
    ratio = max(1, n_s / max(1, n_r))
    rb = 0 if ratio < 2.5 else (1 if ratio < 8 else 2)
    return lr, rb


RATIO_OF_BUCKET = {0: 1, 1: 4, 2: 16}


def measure(c: Candidate, n_r: int, n_s: int, domain: int, reps: int = 5, seed: int = 11) -> float:
    """Mean device time (s) of one hj_join with candidate c (events around the call)."""
    import torch

    from . import hj
    from .gen import device as dgen
    t = dgen.unique_uniform(seed, n_r, n_s, domain)
    p = c.params()
    ws = hj.workspace(p, n_r, n_s)
    out_r = torch.empty(max(1, n_s), dtype=torch.int32, device="cuda")
    out_s = torch.empty_like(out_r)
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    for _ in range(2):
        hj.hj_join(p, *t, out_r, out_s, ws, d)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        hj.hj_join(p, *t, out_r, out_s, ws, d)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps * 1e-3


def tune(log2_r=range(10, 23), ratios=(0, 1, 2), top: int = 4, match: float = 0.625, verbose=True) -> dict:
    """Times the model's best `top` candidates for every bucket; returns the table."""
    table = {"device": "MI355X (gfx950)", "method": "cost-model ranked grid, best measured", "buckets": {}}
    for lr in log2_r:
        for rb in ratios:
            n_r = 1 << lr
            n_s = n_r * RATIO_OF_BUCKET[rb]
            dom = max(n_r, int(math.ceil(n_r / match)))
            m = n_s * n_r / dom
            cands = sorted(candidates(n_r, n_s), key=lambda c: predict(c, n_r, n_s, m))[:top]
            timed = [(measure(c, n_r, n_s, dom), c) for c in cands]
            timed.sort(key=lambda x: x[0])
            best_t, best = timed[0]
            table["buckets"]["%d:%d" % (lr, rb)] = {
                "n_r": n_r, "n_s": n_s, "best": best.as_dict(), "ms": round(best_t * 1e3, 4),
                "timed": [{"cand": c.as_dict(), "ms": round(t_ * 1e3, 4),
                           "model_ms": round(predict(c, n_r, n_s, m) * 1e3, 4)} for t_, c in timed],
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


def choose(n_r: int, n_s: int, table: dict | None) -> Candidate:
    """Tuned candidate for a job (nearest bucket), or the model's pick without a table."""
    if table:
        # from this |R| on, the library's own HJ_AUTO choice (set where timing the
        # whole batch, not single joins, found it faster)
        af = table.get("auto_from_log2")
        if af is not None and n_r >= (1 << int(af)):
            return Candidate("auto", 0)
        lr, rb = bucket_key(n_r, n_s)
        lrs = sorted({int(k.split(":")[0]) for k in table["buckets"]})
        lr = min(lrs, key=lambda x: abs(x - lr))
        e = table["buckets"].get("%d:%d" % (lr, rb))
        if e:
            c = Candidate.from_dict(e["best"])
            if c.algo == "phj" and c.passes == 0 and n_r > 8192:
                c = Candidate("phj", 1, (max(1, _bits_for(n_r)), 0))
            return c
    m = 0.625 * n_s
    return min(candidates(n_r, n_s), key=lambda c: predict(c, n_r, n_s, m))


def main():
    ap = argparse.ArgumentParser(description="tune per-bucket join parameters on the GPU")
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--min-log2", type=int, default=10)
    ap.add_argument("--max-log2", type=int, default=22)
    ap.add_argument("--top", type=int, default=4)
    ap.add_argument("--merge", action="store_true",
                    help="keep the buckets of the existing table outside the tuned range")
    ap.add_argument("--set-auto-from-log2", type=int, default=None, metavar="L",
                    help="no tuning: mark the existing table so jobs with |R| >= 2^L take HJ_AUTO's choice")
    ap.add_argument("--note", default="", help="why (stored with --set-auto-from-log2)")
    a = ap.parse_args()
    if a.set_auto_from_log2 is not None:
        table = load_table(a.out)
        table["auto_from_log2"] = a.set_auto_from_log2
        table["auto_note"] = a.note
        with open(a.out, "w") as f:
            json.dump(table, f, indent=1)
        print(a.out)
        return
    table = tune(range(a.min_log2, a.max_log2 + 1), top=a.top)
    old = load_table(a.out) if a.merge else None
    if old:
        for k, v in old["buckets"].items():
            table["buckets"].setdefault(k, v)
        table["buckets"] = dict(sorted(table["buckets"].items(), key=lambda kv: tuple(map(int, kv[0].split(":")))))
    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1)
    print(a.out)


if __name__ == "__main__":
    main()
