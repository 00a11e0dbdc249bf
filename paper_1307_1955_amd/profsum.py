"""Summaries of rocprofv3 runs of the join kernels (for the profiles/ folder).

Reads the CSV output of
  * one ``rocprofv3 --kernel-trace --stats`` run (per-kernel average duration),
  * one ``--pmc FETCH_SIZE`` and one ``--pmc WRITE_SIZE`` run of the same
    command (KiB per dispatch),
  * the same two counters for a plain device copy of known size,
and writes a short markdown table plus a JSON record.  HBM bytes of a kernel
= counter KiB * 1024 * (copy bytes / copy counter bytes): the copy scales each
counter to true bytes.  The JSON keeps a hash of the kernel sources' code
(comments excluded) so a consumer can tell whether the kernels changed since
the counters were taken.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/phj_partition.hip", "csrc/phj_join.hip", "csrc/shj.hip", "csrc/scan.hip", "csrc/hj_side.h",
                  "csrc/hj_device.h", "csrc/hj_heavy.h", "csrc/hj_internal.h"]


def code_only(text: str) -> str:
    """C/C++ source without its comments, each line stripped and empty lines
    dropped: what the compiler sees, so that edits of comments alone keep the
    hash (string and character literals are kept as they are)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    lines = (" ".join(ln.split()) for ln in "".join(out).splitlines())
    return "\n".join(ln for ln in lines if ln)


def sources_hash() -> str:
    """sha256 over the kernel sources' code (comments excluded)."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(PKG, rel), "r", encoding="utf-8") as f:
            h.update(code_only(f.read()).encode())
    return h.hexdigest()


def short_name(name: str) -> str:
    """"void hj::(anonymous namespace)::k_part_scatter<16u>(...)" -> "k_part_scatter<16u>"."""
    m = re.search(r"(k_[A-Za-z0-9_]+(?:<[^>(]*>)?)\(", name)
    if m:
        return m.group(1)
    return name.split("(")[0].replace("void ", "").strip()


def one_csv(d: str, suffix: str) -> str:
    hits = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not hits:
        raise FileNotFoundError("no *%s under %s" % (suffix, d))
    return hits[0]


def counters(d: str) -> dict:
    acc = collections.defaultdict(list)
    for r in csv.DictReader(open(one_csv(d, "counter_collection.csv"))):
        acc[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def stats(d: str) -> dict:
    out = {}
    for r in csv.DictReader(open(one_csv(d, "kernel_stats.csv"))):
        out[short_name(r["Name"])] = {"calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
                                      "total_ns": float(r["TotalDurationNs"])}
    return out


def sq_table(d: str) -> str:
    """Per-kernel means of one SQ counter pass (SQ_WAVES, SQ_WAVE_CYCLES,
    SQ_WAIT_INST_ANY, SQ_INSTS_VALU, SQ_INSTS_LDS, SQ_LDS_BANK_CONFLICT) as a
    markdown table: waves, VALU and LDS instructions per wave, bank-conflict
    cycles per LDS instruction, share of wave cycles waiting on any instruction."""
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    for r in csv.DictReader(open(one_csv(d, "counter_collection.csv"))):
        k = short_name(r["Kernel_Name"])
        if not k.startswith("k_"):
            continue
        per[(k, r["Dispatch_Id"])][r["Counter_Name"]] += float(r["Counter_Value"])
    agg = collections.defaultdict(list)
    for (k, _), c in per.items():
        agg[k].append(c)
    lines = ["| kernel | waves | VALU / wave | LDS / wave | conflict cycles / LDS instr | wait / wave cycles |",
             "|---|---:|---:|---:|---:|---:|"]
    for k in sorted(agg, key=lambda k: -sum(c.get("SQ_WAVE_CYCLES", 0.0) for c in agg[k])):
        cs = agg[k]

        def mean(n):
            return sum(c.get(n, 0.0) for c in cs) / len(cs)
        w, lds = mean("SQ_WAVES"), mean("SQ_INSTS_LDS")
        if w == 0:
            continue
        lines.append("| %s | %d | %d | %d | %.2f | %.2f |" % (
            k, w, mean("SQ_INSTS_VALU") / w, lds / w, mean("SQ_LDS_BANK_CONFLICT") / lds if lds else 0.0,
            mean("SQ_WAIT_INST_ANY") / max(mean("SQ_WAVE_CYCLES"), 1.0)))
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-bytes", type=int, required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--commands", required=True, help="the commands that produced the CSVs")
    ap.add_argument("--prefix", default="k_", help="only kernels whose name starts with this")
    ap.add_argument("--out-md", required=True)
    ap.add_argument("--out-json", required=True)
    ap.add_argument("--sq", default=None, metavar="DIR",
                    help="a --pmc run of the SQ counters of sq_table(): its table is appended")
    ap.add_argument("--sq-command", default="", help="the command of the --sq run")
    a = ap.parse_args()
    st = stats(a.trace)
    fe, wr = counters(a.fetch), counters(a.write)
    cf, cw = counters(a.copy_fetch), counters(a.copy_write)
    copy_name = max(cf, key=lambda k: cf[k])
    f_factor = a.copy_bytes / (cf[copy_name] * 1024.0)
    w_factor = a.copy_bytes / (cw[copy_name] * 1024.0)
    rows = []
    for k in sorted(st, key=lambda x: -st[x]["total_ns"]):
        if not k.startswith(a.prefix):
            continue
        rows.append({"kernel": k, "calls": st[k]["calls"], "avg_us": st[k]["avg_ns"] / 1e3,
                     "hbm_read_mb": fe.get(k, 0.0) * 1024 * f_factor / 1e6 if k in fe else None,
                     "hbm_write_mb": wr.get(k, 0.0) * 1024 * w_factor / 1e6 if k in wr else None})
    rec = {"workload": a.workload, "commands": a.commands, "copy_kernel": copy_name, "copy_bytes": a.copy_bytes,
           "fetch_factor": f_factor, "write_factor": w_factor, "sources_sha256": sources_hash(), "kernels": rows}
    with open(a.out_json, "w") as f:
        json.dump(rec, f, indent=1)
    lines = ["# rocprofv3: %s" % a.workload, "", "Commands (run from the repository root on an MI355X):", "",
             "```", a.commands, "```", "",
             "HBM bytes = counter KiB x 1024 x factor; factors from a plain %d-byte device copy (%s): "
             "FETCH_SIZE x %.3f, WRITE_SIZE x %.3f." % (a.copy_bytes, copy_name, f_factor, w_factor), "",
             "| kernel | calls | avg us | HBM read MB / dispatch | HBM write MB / dispatch |",
             "|---|---:|---:|---:|---:|"]
    for r in rows:
        fmt = lambda v: "-" if v is None else "%.1f" % v
        lines.append("| %s | %d | %.1f | %s | %s |" % (r["kernel"], r["calls"], r["avg_us"], fmt(r["hbm_read_mb"]),
                                                      fmt(r["hbm_write_mb"])))
    lines.append("")
    lines.append("Kernel sources sha256 at measurement (code without comments): `%s`" % rec["sources_sha256"])
    if a.sq:
        lines += ["", "## SQ counters (one pass of 8)", "", "```", a.sq_command, "```", "",
                  "Per dispatch (means): waves, VALU and LDS instructions per wave, LDS bank-conflict cycles per "
                  "LDS instruction, and the share of wave cycles spent waiting on any instruction.", "",
                  sq_table(a.sq).rstrip()]
    with open(a.out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(a.out_md, a.out_json)


if __name__ == "__main__":
    main()
