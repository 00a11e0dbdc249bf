"""Per-step cost model of a join on MI355X (Section 4, Eq. 2-3), for planning.

The paper's abstract model sums, over the steps of a step series, each step's
computation time, memory-stall time and pipelined delay behind the previous
step, and takes the longer of the two processors.  Here one GPU runs every
step and a step is one kernel launch of the plan (the launch sequence of
csrc/engine.cpp), so

    T = sum over launches k of  D + d + max(M_k, W_k)

with D the delay of a dependent launch (its start behind the previous
kernel's end), d a kernel's fixed ramp-up and drain, M_k the launch's algorithmic bytes over the bandwidth its
access pattern reaches (streaming, scatter by run length, random table
lines), and W_k the latency term of its workgroups: ceil(workgroups / resident
slots) rounds of one workgroup's duration.  The computation term of Eq. 2 is
folded into W_k and into the per-tuple costs of the random-access steps; those
constants, like the bandwidths, are calibrated on the device (``tune.py
--collect`` records per-kernel HIP-event times over a grid of joins, ``fit``
fits each kernel's constants).  The same formulas are compiled into the
library (csrc/costmodel.cpp, constants from tuning/mi355x_calib.json via
tuning/calib_mi355x.inc), where HJ_AUTO evaluates them; a CPU test keeps the
two in agreement.
"""
from __future__ import annotations

import json
import math
import os

PKG = os.path.dirname(os.path.abspath(__file__))
CALIB_JSON = os.path.join(PKG, "tuning", "mi355x_calib.json")
CALIB_INC = os.path.join(PKG, "csrc", "calib_mi355x.inc")

CUS = 256
LDS_PER_CU = 160 * 1024
JOIN_CHUNK = 9216          # S tuples per join work item
OVF_CHUNK = 2048           # R tuples per HBM-table build item,
OVF_CHUNK_BIG = 16384      #   in a partition of more than OVF_BIG_PART tuples
OVF_BIG_PART = 1 << 16
OVF_GRID = 2048            # workgroups of the HBM-table build launches
SHJ_TILE = 2048            # S tuples per SHJ probe workgroup
SCAN_CHUNK = 2048          # entries per scan workgroup
COUNTED_MAX_BITS = 13      # two passes of 4..13 bits in all: pass 1 counts the final partitions

# the fitted constants, in this order (seconds, bytes/s; positive except SIGNED)
PARAMS = [
    "d_gap",               # delay of a dependent launch behind the previous kernel
    "d_kernel",            # fixed ramp-up and drain of a kernel
    "bw_hist", "t_hist_tile",
    "t_count_bin",         # a counted pass 2's histogram tile: clear, count and pack 2^bits counters
    "bw_scatter", "run_half", "t_scatter_tile",
    "t_reserve",           # a counted pass 2's scatter tile: count sums beside it, or reservations
    "p_part",              # the partitioning kernels overlap memory and latency imperfectly: (M^p + W^p)^(1/p)
    "q_part",              # share of a later round of partitioning tiles whose latency shows (rounds overlap)
    "t_scan_entry",
    "bw_join", "l_join0", "l_join_r", "l_join_s",
    "f_count", "f_1pass",  # a work item's latency in the count pass and the one-pass write, against the write pass
    "p_join",              # the join kernels overlap memory and latency imperfectly: (M^p + W^p)^(1/p)
    "l_hbm0", "l_hbm_s", "t_ovf_insert", "l_ovf_round",
    "bw_fill",
    # random table accesses: throughput n * t * (table MiB)^gamma, at least a
    # latency floor t_round * (table / 32 KiB)^gamma_round (one round of
    # dependent accesses per resident lane, slower as fewer lines hit the caches)
    "t_ins", "gamma_ins", "t_bround", "gamma_bround",
    "t_probe", "gamma_probe", "t_pround", "gamma_pround", "t_match",
]
# may be negative: back-to-back launches overlap (d_gap); the per-access cost
# may fall with the table size while the chip fills (the exponents)
SIGNED = {"d_gap", "gamma_ins", "gamma_bround", "gamma_probe", "gamma_pround"}


def load(path: str = CALIB_JSON) -> dict:
    with open(path) as f:
        return json.load(f)["params"]


SHJ_SLOTS_PER_ROW = 2.0  # csrc/hj_internal.h kShjSlotsPerRow


def shj_slots(n_r: int) -> int:
    s = int(SHJ_SLOTS_PER_ROW * max(n_r, 1) + 0.999999)
    return (s + 15) // 16 * 16


def _part_block(tile: int) -> int:
    return 512 if tile >= 4096 else 256


def _scatter_slots(bits: int, tile: int) -> int:
    P = 1 << bits
    Pp = max(P, 64)
    lds = 4 * (2 * Pp + 16) + 8 * tile
    by_lds = LDS_PER_CU // lds
    by_threads = 2048 // _part_block(tile)
    return CUS * max(1, min(by_lds, by_threads))


def _hist_slots(tile: int) -> int:
    return CUS * (2048 // _part_block(tile))


def join_lds_bytes(cap: int) -> int:
    return 4 * (cap + 128) + 8 * cap


def join_slots(cap: int) -> int:
    """Join work items resident at once: workgroups per CU by LDS and by the
    waves the kernels' register budget allows (6 per SIMD, 4 with the largest
    build), 512-thread workgroups."""
    by_waves = (4 if cap > 4608 else 6) * 4 // 8
    return CUS * max(1, min(LDS_PER_CU // (join_lds_bytes(cap) + 1024), by_waves))


def _nonempty(mean: float) -> float:
    return 1.0 - math.exp(-mean) if mean < 30 else 1.0


def _smooth_max(a: float, b: float, p: float) -> float:
    """(a^p + b^p)^(1/p): max(a, b) as p grows, more than it when a and b are close."""
    m = max(a, b)
    if m <= 0.0:
        return 0.0
    return m * ((a / m) ** p + (b / m) ** p) ** (1.0 / p)


def _table_factor(table_bytes: float, gamma: float, base: float = 1 << 20) -> float:
    """Change of a random access's cost with the table size (1 up to base bytes)."""
    return (max(table_bytes, base) / base) ** gamma


def counted_pass2(passes: int, b1: int, b2: int) -> bool:
    """Two passes whose pass 2 reserves its runs on counts taken in pass 1."""
    return passes == 2 and 4 <= b1 + b2 <= COUNTED_MAX_BITS


def launches(plan: dict, n_r: int, n_s: int, m: float) -> list[tuple[str, dict]]:
    """The launch sequence of a join (engine.cpp) with each launch's features.
    plan: resolved parameters: algo ("shj"/"phj"), passes, bits (b1, b2), tile,
    lds_cap, one_pass."""
    n = n_r + n_s
    out = []
    if n_r == 0 or n_s == 0:
        return [("zero_count", {})]
    if plan["algo"] == "shj":
        slots = shj_slots(n_r)
        tb = 8.0 * slots
        out.append(("shj_fill", {"bytes": 8.0 * slots}))
        out.append(("shj_build", {"n": n_r, "tb": tb}))
        if plan["one_pass"]:
            out.append(("zero_count", {}))
            out.append(("shj_write_1pass", {"n": n_s, "tb": tb, "m": m}))
        else:
            tiles = math.ceil(n_s / SHJ_TILE)
            out.append(("shj_count", {"n": n_s, "tb": tb}))
            out.append(("zero_state", {}))
            out.append(("scan_u64", {"entries": 4 * tiles}))
            out.append(("shj_write", {"n": n_s, "tb": tb, "m": m}))
        return out
    cap = plan["lds_cap"]
    if plan["passes"] == 0:
        items = math.ceil(n_s / JOIN_CHUNK)
        out.append(("direct_setup", {}))
        out.append(("direct_join", {"items": items, "grid": items, "r": n_r, "s": min(n_s, JOIN_CHUNK), "cap": cap,
                                    "bytes": 8.0 * n + 8.0 * m, "hbm": 0}))
        return out
    tile = plan["tile"]
    b1, b2 = plan["bits"][0], (plan["bits"][1] if plan["passes"] == 2 else 0)
    B = b1 + b2
    P = 1 << B
    P1 = 1 << b1
    tiles1 = math.ceil(n_r / tile) + math.ceil(n_s / tile)
    counted = counted_pass2(plan["passes"], b1, b2)
    rows = float(tiles1 * P) if counted else 0.0  # 8-bit count rows: written by the histogram, summed beside the scatter
    out.append(("part_hist", {"n": n, "tiles": tiles1, "tile": tile, "extra": rows, "bins": P if counted else 0}))
    out.append(("scan_u32", {"entries": tiles1 * P1}))
    out.append(("part_scatter", {"n": n, "tiles": tiles1, "tile": tile, "bits": b1, "extra": rows,
                                 "counted": int(counted)}))
    r_part, s_part = n_r / P, n_s / P
    hbm = r_part > cap
    ovf_r = n_r if hbm else 0
    # a counted pass 2 of at most 64 partitions per segment clears the HBM tables itself
    clears = counted and b2 <= 6
    if plan["passes"] == 2:
        seg = n / (2.0 * P1)
        tiles2 = 2 * P1 * max(1, math.ceil(seg / tile)) if seg > 0 else 0
        if not counted:
            out.append(("part_hist", {"n": n, "tiles": tiles2, "tile": tile, "extra": 0.0, "bins": 0}))
            out.append(("scan_u32", {"entries": (n / tile + 2 * P1) * (1 << b2)}))
        out.append(("part_scatter", {"n": n, "tiles": tiles2, "tile": tile, "bits": b2,
                                     "extra": 16.0 * ovf_r if clears else 0.0, "counted": int(counted)}))
    pairs = P * _nonempty(r_part) * _nonempty(s_part)
    items = pairs * max(1, math.ceil(s_part / JOIN_CHUNK))
    grid = P + math.ceil(n_s / JOIN_CHUNK)
    s_item = min(max(s_part, 1.0), JOIN_CHUNK)
    chunk = OVF_CHUNK_BIG if r_part > OVF_BIG_PART else OVF_CHUNK
    ovf_items = P * math.ceil(r_part / chunk) if hbm else 0
    if not clears:
        out.append(("ovf_clear", {"bytes": 16.0 * ovf_r}))
    out.append(("ovf_build", {"n": ovf_r, "items": ovf_items, "per": min(r_part, chunk)}))
    jf = {"items": items, "grid": grid, "r": min(r_part, cap), "s": s_item, "cap": cap, "hbm": int(hbm)}
    if not plan["one_pass"]:
        out.append(("join_count", dict(jf, bytes=4.0 * n)))
        out.append(("scan_u64", {"entries": 8 * grid}))
        out.append(("join_write", dict(jf, bytes=8.0 * n + 8.0 * m)))
    else:
        out.append(("join_write_1pass", dict(jf, bytes=8.0 * n + 8.0 * m)))
    return out


def _part_lat(rounds: int, per_tile: float, c: dict) -> float:
    """Latency term of a partitioning launch: the first round of tiles, then a
    share q_part of each later round (rounds overlap)."""
    return per_tile * (1.0 + (rounds - 1) * c["q_part"])


def kernel_seconds(name: str, f: dict, c: dict) -> float:
    """One kernel's duration: ramp-up/drain + max(memory term, workgroup-latency term)."""
    d = c["d_kernel"]
    if name == "part_hist":
        if f["tiles"] == 0:
            return d
        rounds = math.ceil(f["tiles"] / _hist_slots(f["tile"]))
        per_tile = c["t_hist_tile"] * f["tile"] / 8192.0 + c["t_count_bin"] * f["bins"]
        return d + _smooth_max((4.0 * f["n"] + f["extra"]) / c["bw_hist"], _part_lat(rounds, per_tile, c),
                               c["p_part"])
    if name == "part_scatter":
        if f["tiles"] == 0:
            return d
        run = f["tile"] / float(1 << f["bits"])
        bw = c["bw_scatter"] * run / (run + c["run_half"])
        rounds = math.ceil(f["tiles"] / _scatter_slots(f["bits"], f["tile"]))
        per_tile = c["t_scatter_tile"] * f["tile"] / 8192.0 + c["t_reserve"] * f["counted"]
        return d + _smooth_max((16.0 * f["n"] + f["extra"]) / bw, _part_lat(rounds, per_tile, c), c["p_part"])
    if name in ("scan_u32", "scan_u64"):
        return d + f["entries"] * c["t_scan_entry"]
    if name in ("join_count", "join_write", "join_write_1pass", "direct_join"):
        if f["hbm"]:
            lat = c["l_hbm0"] + c["l_hbm_s"] * f["s"]
        else:
            lat = c["l_join0"] + c["l_join_r"] * f["r"] + c["l_join_s"] * f["s"]
        lat *= c["f_count"] if name == "join_count" else c["f_1pass"] if name == "join_write_1pass" else 1.0
        rounds = math.ceil(max(f["items"], 1) / join_slots(f["cap"]))
        return d + _smooth_max(f["bytes"] / c["bw_join"], rounds * lat, c["p_join"])
    if name == "ovf_clear":
        return d + f["bytes"] / c["bw_fill"]
    if name == "ovf_build":
        if not f["items"]:
            return d
        rounds = math.ceil(f["items"] / min(OVF_GRID, 8 * CUS))
        return d + max(f["n"] * c["t_ovf_insert"], rounds * math.ceil(f["per"] / 256.0) * c["l_ovf_round"])
    if name == "shj_fill":
        return d + f["bytes"] / c["bw_fill"]
    if name == "shj_build":
        floor = c["t_bround"] * _table_factor(f["tb"], c["gamma_bround"], 32768.0)
        return d + max(f["n"] * c["t_ins"] * _table_factor(f["tb"], c["gamma_ins"]), floor)
    if name in ("shj_count", "shj_write", "shj_write_1pass"):
        t = f["n"] * c["t_probe"] * _table_factor(f["tb"], c["gamma_probe"])
        if name != "shj_count":
            t += f["m"] * c["t_match"]
        return d + max(t, c["t_pround"] * _table_factor(f["tb"], c["gamma_pround"], 32768.0))
    return d  # small set-up kernels: the delay alone


def join_seconds(plan: dict, n_r: int, n_s: int, m: float, c: dict) -> float:
    ls = launches(plan, n_r, n_s, m)
    return sum(kernel_seconds(k, f, c) for k, f in ls) + len(ls) * c["d_gap"]


# starting point of the fit: rough MI355X figures
START = {
    "d_gap": 2e-6, "d_kernel": 3e-6, "bw_hist": 4.5e12, "t_hist_tile": 5e-6, "t_count_bin": 1e-9,
    "bw_scatter": 5.2e12, "run_half": 8.0, "t_scatter_tile": 12e-6, "t_reserve": 2e-6, "p_part": 4.0, "q_part": 0.5, "t_scan_entry": 2e-12, "bw_join": 4e12, "l_join0": 4e-6, "l_join_r": 1e-9,
    "l_join_s": 5e-10, "f_count": 0.8, "f_1pass": 1.2, "p_join": 4.0, "l_hbm0": 8e-6, "l_hbm_s": 2e-9, "t_ovf_insert": 1e-10, "l_ovf_round": 4e-6,
    "bw_fill": 5e12, "t_ins": 1e-10, "gamma_ins": -0.2, "t_bround": 1e-5, "gamma_bround": 0.1,
    "t_probe": 3e-11, "gamma_probe": 0.0, "t_pround": 2e-5, "gamma_pround": 0.1, "t_match": 1e-11,
}


def fit(raw: dict) -> tuple[dict, dict]:
    """Fits the constants to per-kernel HIP-event times (``tune.py --collect``
    records): least squares on log(predicted / measured) over every launch, then
    the launch gap from the whole-join times.  Returns (params, fit report)."""
    import numpy as np
    from scipy.optimize import least_squares

    pts = []  # (kernel name, features, measured seconds)
    joins = []  # (launch list, measured kernel seconds list, whole join seconds)
    for r in raw["records"]:
        rs = r["resolved"]
        plan = {"algo": "shj" if rs["algo"] == 0 else "phj", "passes": rs["passes"], "bits": tuple(rs["bits"]),
                "tile": rs["tile"], "lds_cap": rs["lds_cap"], "one_pass": rs["one_pass"]}
        ls = launches(plan, r["cfg"]["n_r"], r["cfg"]["n_s"], r["pairs"])
        names = [k for k, _ in r["kernels"]]
        if names != [k for k, _ in ls]:
            raise ValueError("launch sequence of %r: recorded %s, modelled %s" % (r["cfg"], names, [k for k, _ in ls]))
        for (k, f), (_, ms) in zip(ls, r["kernels"]):
            pts.append((k, f, max(ms, 1e-4) * 1e-3))
        joins.append((plan, r["cfg"]["n_r"], r["cfg"]["n_s"], r["pairs"], r["join_ms"] * 1e-3, len(ls)))
    free = [k for k in PARAMS if k != "d_gap"]
    signed = [k in SIGNED for k in free]

    def params_of(x):
        c = {k: float(v if sg else np.exp(v)) for k, v, sg in zip(free, x, signed)}
        c["d_gap"] = 0.0
        return c

    def x_of(c):
        return np.array([c[k] if sg else math.log(c[k]) for k, sg in zip(free, signed)])

    def resid(x):
        c = params_of(x)
        return np.array([math.log(kernel_seconds(k, f, c) / t) for k, f, t in pts])

    sol = least_squares(resid, x_of(START), method="trf", max_nfev=4000)
    c = params_of(sol.x)
    # the launch gap: what whole joins take beyond their kernels' event times
    gaps = [(t - sum(kernel_seconds(k, f, c) for k, f in launches(plan, nr, ns, m))) / nl
            for plan, nr, ns, m, t, nl in joins]
    c["d_gap"] = float(np.median(gaps))
    r = resid(sol.x)
    err = [join_seconds(plan, nr, ns, m, c) / t - 1.0 for plan, nr, ns, m, t, nl in joins]
    report = {"launches": len(pts), "joins": len(joins),
              "kernel_abs_log_err_median": float(np.median(np.abs(r))),
              "kernel_abs_log_err_p90": float(np.percentile(np.abs(r), 90)),
              "join_abs_rel_err_median": float(np.median(np.abs(err))),
              "join_abs_rel_err_p90": float(np.percentile(np.abs(err), 90)),
              "join_within_15pct": float(np.mean(np.abs(err) <= 0.15))}
    return {k: c[k] for k in PARAMS}, report


def plan_of(resolved) -> dict:
    """Plan dict from a resolved HjParams (hj_resolve_params)."""
    return {"algo": "shj" if resolved.algo == 0 else "phj", "passes": int(resolved.passes),
            "bits": (int(resolved.bits[0]), int(resolved.bits[1])), "tile": int(resolved.tile),
            "lds_cap": int(resolved.lds_cap), "one_pass": bool(resolved.flags & 1)}


def write_inc(params: dict, path: str = CALIB_INC) -> None:
    """The constants as a C++ include for csrc/costmodel.cpp (generated; do not edit)."""
    lines = ["// Generated by paper_1307_1955_amd.costmodel.write_inc from tuning/mi355x_calib.json;",
             "// the per-step cost model's constants calibrated on MI355X.  Do not edit."]
    for k in PARAMS:
        lines.append("constexpr double k_%s = %.17g;" % (k, params[k]))
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
