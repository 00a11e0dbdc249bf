#!/usr/bin/env python3
"""Benchmark of the hash join hot path on one MI355X.

A step is one PHJ join of the 16M x 16M workload (R keys a permutation of
1..2^24, S keys uniform over 1..2^25, so about half of S matches), inputs
resident in HBM before timing starts, output materialised in HBM.  Prints one
JSON line: input tuples/s of PHJ (the headline value), the same for SHJ on the
same inputs, per-kernel times and the roofline of the dominant kernel
(algorithmic bytes / HIP-event duration, against 8 TB/s), and the CPU oracle
timed on the host as a reference point.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "input tuples/s, SHJ & PHJ 16M⋈16M; batched joins/s; p50/p99 latency at fixed QPS"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--passes", type=int, default=2)
    ap.add_argument("--bits", type=str, default="6,6")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--hash", type=str, default="identity", choices=["identity", "murmur2"])
    ap.add_argument("--n", type=int, default=1 << 24, help="|R| = |S| (default 2^24)")
    ap.add_argument("--two-pass", action="store_true",
                    help="headline PHJ with the two-pass output (count, scan, write) instead of one-pass")
    ap.add_argument("--no-shj", action="store_true", help="skip the SHJ line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweeps", action="store_true",
                    help="skip the radix sweep of the 16M x 16M workload (6-14 bits over one or two passes) and the "
                         "build-size (|R| 2^16..2^24 against |S| = 2^24), selectivity (12.5/50/100%% of S "
                         "matching) and skew-set sweeps that the default run times")
    ap.add_argument("--no-c3", action="store_true", help="skip the Zipf-skewed 16M x 64M workload and the skewed-R sets")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the 16M x 16M PHJ and SHJ lines (no build/probe, no C3), e.g. under a profiler")
    ap.add_argument("--batch-jobs", type=int, default=4096, help="jobs of the batched workload (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--serve-requests", type=int, default=12288, help="requests per served level (0: skip)")
    ap.add_argument("--serve-warmup", type=int, default=2048)
    ap.add_argument("--serve-slots", type=int, default=16, help="concurrent batches of the server (1..16)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates the HBM byte counters)")
    return ap.parse_args()


def algorithmic_bytes(name: str, n_r: int, n_s: int, m: int) -> float | None:
    """Bytes a launch of `name` must move (SoA int32 keys and rids)."""
    n = n_r + n_s
    return {
        "part_hist": 4.0 * n,            # read keys
        "part_scatter": 16.0 * n,        # read key+rid, write key+rid
        "join_count": 4.0 * n,           # read R_i and S_i keys
        "join_write": 8.0 * n + 8.0 * m,  # read key+rid of R_i and S_i, write the pairs
        "join_write_1pass": 8.0 * n + 8.0 * m,
        "shj_build": 4.0 * n_r,          # read R keys (table traffic is random, counted separately)
        "shj_count": 4.0 * n_s,
        "shj_write": 8.0 * n_s + 8.0 * m,
        "shj_write_1pass": 8.0 * n_s + 8.0 * m,
    }.get(name)


CLOCK_RAMP_MS = 30.0  # untimed work before the warm-up steps of the headline join


def clock_ramp(fn, torch, min_ms: float = CLOCK_RAMP_MS) -> float:
    """Runs fn (untimed) until at least min_ms of device time has passed, so the
    GPU's clocks are at their steady level when the warm-up steps begin (the
    same rule as the calibration's steady timing).  Returns the time spent."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < min_ms:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3


def time_steps(fn, steps: int, warmup: int, torch) -> float:
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def kernel_times(hj, p, t, out_r, out_s, ws, d_count, reps: int):
    """Average HIP-event duration of each kernel over `reps` timed joins."""
    acc: dict[str, list[float]] = {}
    for _ in range(reps):
        for name, ms in hj.hj_join_timed(p, *t, out_r, out_s, ws, d_count):
            acc.setdefault(name, []).append(ms)
    return acc


def summarize(acc, reps, n_r, n_s, m):
    rows = {}
    for name, v in acc.items():
        per_join = sum(v) / reps
        launches = len(v) / reps
        avg = sum(v) / len(v)
        ab = algorithmic_bytes(name, n_r, n_s, m)
        row = {"ms_per_join": round(per_join, 4), "launches_per_join": launches, "avg_launch_ms": round(avg, 4)}
        if ab is not None:
            # algorithmic bytes of one launch: passes launch the kernel once each
            row["gbs"] = round(ab / (avg * 1e-3) / 1e9, 1)
        rows[name] = row
    return rows


def bench_batched(args, torch, hj, wl, params, table) -> dict:
    """4096 joins of log-uniform sizes: one graph-captured batch vs plain per-join calls.
    After the timed runs every job is checked on the device (count = closed form,
    every pair joins equal keys, no S row twice)."""
    from paper_1307_1955_amd import workloads
    plan = hj.BatchPlan(wl.jobs, wl.d_counts, params=params)
    ws = plan.workspace()
    expected = torch.tensor(wl.expected, dtype=torch.int64, device="cuda")
    print("bench: batch plan: %d direct jobs, workspace %.2f GB; capturing the graph" % (
        plan.direct_jobs, plan.workspace_bytes / 1e9), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    plan.run(ws)
    torch.cuda.synchronize()
    first_s = time.perf_counter() - t0
    ok = bool(torch.equal(wl.d_counts, expected))
    ms = time_steps(lambda: plan.run(ws), args.batch_steps, 0, torch)
    ok = ok and bool(torch.equal(wl.d_counts, expected))
    # the same jobs through plain per-join calls on one stream, one workspace
    print("bench: plain per-join path", file=sys.stderr, flush=True)
    ws_one = torch.empty(max(hj.hj_workspace_bytes(q, sp.n_r, sp.n_s) for q, sp in zip(params, wl.specs)),
                         dtype=torch.uint8, device="cuda")
    d_one = torch.zeros(1, dtype=torch.int64, device="cuda")
    one_counts = torch.zeros(len(wl.jobs), dtype=torch.int64, device="cuda")

    def plain():
        for j, (job, q) in enumerate(zip(wl.jobs, params)):
            hj.hj_join(q, *job, ws_one, one_counts[j:j + 1])

    print("bench: checking every batched job on the device", file=sys.stderr, flush=True)
    bad = workloads.verify_device(wl)
    ms_plain = time_steps(plain, 1, 1, torch)
    same = bool(torch.equal(one_counts, expected))
    del d_one
    res = {
        "metric": "joins/s", "value": len(wl.jobs) / (ms * 1e-3), "jobs": len(wl.jobs), "ms_per_batch": ms,
        "tuples_per_s": wl.tuples / (ms * 1e-3),
        "config": "4096 joins, |R| log-uniform in [1024, 4194304], |S| = |R| x U{1..16}, 25-100%% match; "
                  "sum |R|+|S| = %d tuples, %d pairs" % (wl.tuples, wl.pairs),
        "params": "tuning table" if table else "cost model",
        "direct_jobs": plan.direct_jobs, "graph": True, "graph_nodes": plan.graph_nodes,
        "first_run_s_incl_capture": round(first_s, 3),
        "counts_match_closed_form": ok,
        "pairs_verified_on_device": not bad, "failed_jobs": bad[:8],
        "plain_per_join": {"value": len(wl.jobs) / (ms_plain * 1e-3), "ms": ms_plain,
                           "counts_match_closed_form": same},
        "speedup_vs_plain": ms_plain / ms,
    }
    plan.close()
    del ws, ws_one
    torch.cuda.empty_cache()
    return res


def percentile(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def bench_served(args, torch, hj, wl, params, qps_levels) -> dict:
    """Open-loop Poisson arrivals of requests drawn from the batched workload,
    served with continuous batching under a 64 GiB footprint cap, against the
    same trace through plain per-join calls run serially.

    Request i joins job i mod 4096 into that job's output buffer; every request
    has a count slot of its own.  Checked after each level: every request's
    status and count, that no two requests of one job were on the device at
    the same time (so none could overwrite another's pairs), and every job's
    pairs (those of its last request) on the device."""
    import ctypes

    from paper_1307_1955_amd import gen, workloads
    njobs = len(wl.jobs)
    n = args.serve_requests
    warm = min(args.serve_warmup, n // 2)
    ws_max = max(hj.hj_workspace_bytes(q, sp.n_r, sp.n_s) for q, sp in zip(params, wl.specs))
    slots = args.serve_slots
    pool = torch.empty(slots * (ws_max + (64 << 20)), dtype=torch.uint8, device="cuda")
    req_counts = torch.zeros(n, dtype=torch.int64, device="cuda")
    plain_counts = torch.zeros(n, dtype=torch.int64, device="cuda")
    base = req_counts.data_ptr()
    jobs = [hj.make_job(*wl.jobs[i % njobs], base + 8 * i) for i in range(n)]
    fps = [8 * (sp.n_r + sp.n_s) + 8 * e + hj.hj_workspace_bytes(q, sp.n_r, sp.n_s)
           for sp, e, q in zip(wl.specs, wl.expected, params)]
    want = torch.tensor([wl.expected[i % njobs] for i in range(n)], dtype=torch.int64, device="cuda")
    asked = [j for j in range(njobs) if j < n]  # jobs with at least one request
    last = [max(range(j, n, njobs)) for j in asked]  # each one's last request
    lib = hj.load()
    out = {"requests": n, "warmup_requests": warm, "cap_bytes": 64 << 30, "slots": slots, "levels": []}
    for qps in qps_levels:
        arr = gen.poisson_arrivals(17, n, qps)
        sv = hj.Server(pool, mem_cap_bytes=64 << 30, slots=slots, max_batch_jobs=64)
        ticket = ctypes.c_uint64(0)
        lag = []
        submit_t = [0.0] * n
        req_counts.fill_(-1)
        torch.cuda.synchronize()
        print("bench: serving %d requests at %.0f/s" % (n, qps), file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        for i in range(n):
            target = t0 + arr[i]
            while time.perf_counter() < target:
                pass
            now = time.perf_counter()
            j = i % njobs
            st = lib.hj_server_submit(sv._h, ctypes.byref(jobs[i]), ctypes.byref(params[j]), fps[j],
                                      ctypes.byref(ticket))
            if st != 0:
                raise RuntimeError("submit failed: %s" % lib.hj_last_error().decode())
            submit_t[i] = now - t0
            lag.append(now - target)
        sv.drain()
        done = sv.poll(n + 16)
        stats = sv.stats()
        sv.close()
        by_ticket = {t: (s_, lat, q_) for t, s_, lat, q_ in done}
        # tickets are issued 1..n in submission order
        lat = [by_ticket[i + 1][1] for i in range(warm, n)]
        ends = [submit_t[i] + by_ticket[i + 1][1] for i in range(n)]
        span = max(ends[warm:]) - arr[warm]
        statuses_ok = all(by_ticket[i + 1][0] == 0 for i in range(n))
        counts_ok = bool(torch.equal(req_counts, want))
        # a request's end (submission + latency, the server's clock starts a few
        # microseconds later) 1 ms before the next request of its job is submitted
        overlaps = sum(1 for i in range(njobs, n) if ends[i - njobs] + 1e-3 > submit_t[i])
        print("bench: checking every job's pairs on the device", file=sys.stderr, flush=True)
        last_counts = torch.full((njobs,), -1, dtype=torch.int64, device="cuda")
        last_counts[torch.tensor(asked, device="cuda")] = req_counts[torch.tensor(last, device="cuda")]
        bad = workloads.verify_device(wl, counts=last_counts, jobs=asked) if overlaps == 0 else [(-1, "overlap")]
        # the same trace through plain per-join calls, one at a time
        print("bench: plain per-join serial path at %.0f/s" % qps, file=sys.stderr, flush=True)
        ws_one = pool[: ws_max]
        lat_plain = []
        h = ctypes.c_uint64(0)
        plain_counts.fill_(-1)
        t0 = time.perf_counter()
        for i in range(n):
            target = t0 + arr[i]
            while time.perf_counter() < target:
                pass
            j = i % njobs
            st = lib.hj_join_sync(ctypes.byref(params[j]), ctypes.byref(jobs[i].R), ctypes.byref(jobs[i].S),
                                  ctypes.byref(jobs[i].out), ws_one.data_ptr(), ws_max, plain_counts.data_ptr() + 8 * i,
                                  ctypes.byref(h), torch.cuda.current_stream().cuda_stream)
            if st != 0:
                raise RuntimeError("plain join failed: %s" % lib.hj_last_error().decode())
            if i >= warm:
                lat_plain.append(time.perf_counter() - target)
        span_plain = time.perf_counter() - (t0 + arr[warm])
        plain_ok = bool(torch.equal(plain_counts, want))
        out["levels"].append({
            "offered_qps": qps,
            "p50_ms": percentile(lat, 50) * 1e3, "p99_ms": percentile(lat, 99) * 1e3,
            "throughput_joins_per_s": (n - warm) / span,
            "batches": stats["batches"], "rejected": stats["rejected"],
            "max_submit_lag_ms": max(lag) * 1e3,
            "all_ok": statuses_ok and counts_ok and overlaps == 0 and not bad,
            "checks": {"statuses_ok": statuses_ok, "every_request_count_ok": counts_ok,
                       "same_job_overlaps": overlaps, "pairs_verified_on_device": not bad,
                       "failed_jobs": bad[:8]},
            "plain_serial": {"p50_ms": percentile(lat_plain, 50) * 1e3, "p99_ms": percentile(lat_plain, 99) * 1e3,
                             "throughput_joins_per_s": (n - warm) / span_plain, "counts_ok": plain_ok},
        })
        print("bench: served %s" % out["levels"][-1], file=sys.stderr, flush=True)
    del pool
    torch.cuda.empty_cache()
    return out


def cpu_baseline(n: int, min_seconds: float = 10.0, max_reps: int = 6) -> dict:
    """The oracle (single-threaded chained hash join) on the full 16M x 16M
    inputs, repeated until about `min_seconds` of CPU work has been timed."""
    import oracle
    from paper_1307_1955_amd import gen
    r, s = gen.config_c2(n=n)
    times = []
    pairs = 0
    while len(times) < max_reps and sum(times) < min_seconds:
        t0 = time.perf_counter()
        with oracle.Table(r.key, r.rid) as tb:
            o_r, o_s = tb.probe(s.key, s.rid)
        times.append(time.perf_counter() - t0)
        pairs = len(o_r)
    el = sum(times) / len(times)
    return {"value": (len(r) + len(s)) / el, "unit": "tuples/s", "cores": 1, "kind": "oracle",
            "sample": "%d full %d x %d joins (build + probe + emit %d pairs), %.2f s each on average"
                      % (len(times), len(r), len(s), pairs, el), "host": host_cpu()}


def host_cpu() -> str:
    """The host CPU model and logical CPU count, for the CPU baseline record."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return "%s, %d logical CPUs (%d usable here)" % (model or "unknown CPU", os.cpu_count() or 0, host_threads())


def host_threads() -> int:
    """Host threads this process may use (its CPU affinity, capped by
    OMP_NUM_THREADS when that is set)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cap = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return max(1, min(n, cap) if cap > 0 else n)


def cpu_baseline_all_cores(n: int, min_seconds: float = 10.0, max_reps: int = 6) -> dict:
    """The oracle with its probe split over S chunks on every host thread
    (single-threaded build, then a concurrent read-only probe), 16M x 16M."""
    import oracle
    from paper_1307_1955_amd import gen
    r, s = gen.config_c2(n=n)
    threads = host_threads()
    times, build = [], []
    pairs = 0
    while len(times) < max_reps and sum(times) < min_seconds:
        t0 = time.perf_counter()
        with oracle.Table(r.key, r.rid) as tb:
            t1 = time.perf_counter()
            o_r, o_s = tb.probe_threads(s.key, s.rid, threads)
        times.append(time.perf_counter() - t0)
        build.append(t1 - t0)
        pairs = len(o_r)
    el = sum(times) / len(times)
    return {"value": (len(r) + len(s)) / el, "unit": "tuples/s", "cores": threads, "kind": "oracle",
            "sample": "%d full %d x %d joins on %d threads (single-threaded build %.2f s, then the probe split "
                      "over S; %d pairs), %.2f s each on average"
                      % (len(times), len(r), len(s), threads, sum(build) / len(build), pairs, el),
            "host": host_cpu()}


def measure_phj(hj, torch, p, t, out_r, out_s, d_count, n_r, n_s, steps, warmup, passes, one_pass):
    """Throughput of one PHJ configuration plus its per-kernel breakdown."""
    ws = hj.workspace(p, n_r, n_s)
    ramp_ms = clock_ramp(lambda: hj.hj_join(p, *t, out_r, out_s, ws, d_count), torch)
    ms = time_steps(lambda: hj.hj_join(p, *t, out_r, out_s, ws, d_count), steps, warmup, torch)
    m = int(d_count.item())
    reps = 5
    phases = summarize(kernel_times(hj, p, t, out_r, out_s, ws, d_count, reps), reps, n_r, n_s, m)
    # partition passes 20 B/tuple each (histogram read + scatter read and write), less the histogram read of a
    # counted pass 2 (its counts come from pass 1); join: count pass 4 B/tuple (two-pass output) + write pass
    # 8 B/tuple
    from paper_1307_1955_amd import costmodel
    counted = costmodel.counted_pass2(passes, int(p.bits[0]), int(p.bits[1]) if passes == 2 else 0)
    total_bytes = (20.0 * passes - (4.0 if counted else 0.0) + (8.0 if one_pass else 12.0)) * (n_r + n_s) + 8.0 * m
    del ws
    return {"ms": ms, "value": (n_r + n_s) / (ms * 1e-3), "matches": m, "kernels": phases, "clock_ramp_ms": round(ramp_ms, 1),
            "path_gbs": round(total_bytes / (ms * 1e-3) / 1e9, 1),
            "path_frac": round(total_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def bench_build_probe(hj, torch, p, t, out_r, out_s, d_count, steps, warmup) -> dict:
    """The split join on the same inputs: R's table built once (hj_build), then
    S probed against it (hj_probe); a probe partitions only S."""
    rk, rr, sk, sr = t
    tab_ws = torch.empty(hj.hj_table_bytes(p, rk.numel()), dtype=torch.uint8, device=rk.device)
    build_ms = time_steps(lambda: hj.hj_build(p, rk, rr, tab_ws), steps, warmup, torch)
    tab = hj.hj_build(p, rk, rr, tab_ws)
    pws = torch.empty(hj.hj_probe_workspace_bytes(tab, sk.numel()), dtype=torch.uint8, device=rk.device)
    probe_ms = time_steps(lambda: hj.hj_probe(tab, sk, sr, out_r, out_s, pws, d_count), steps, warmup, torch)
    return {"params": repr(tab.params), "build_ms": round(build_ms, 4), "probe_ms": round(probe_ms, 4),
            "build_tuples_per_s": rk.numel() / (build_ms * 1e-3), "probe_tuples_per_s": sk.numel() / (probe_ms * 1e-3),
            "matches": int(d_count.item())}


def device_count(torch, rk, sk) -> int:
    """Pairs the join must produce (sum over S of the R rows with its key), with
    plain PyTorch on the device; generated keys are non-negative."""
    hi = int(max(int(rk.max()), int(sk.max()))) + 1
    cnt = torch.bincount(rk.long(), minlength=hi)
    return int(cnt[sk.long()].sum())


def timed_join(hj, torch, q, t, o_r, o_s, d, steps, warmup, want, dev):
    """Mean time of one join with parameters q; raises if its count is not `want`."""
    n_r, n_s = t[0].numel(), t[2].numel()
    ws = hj.workspace(q, n_r, n_s, dev)
    ms = time_steps(lambda: hj.hj_join(q, *t, o_r, o_s, ws, d), steps, warmup, torch)
    m = int(d.item())
    hj.hj_workspace_status(ws)
    if m != want:
        raise AssertionError("%r: %d pairs, the closed form says %d" % (q, m, want))
    del ws
    return {"ms": round(ms, 4), "tuples_per_s": (n_r + n_s) / (ms * 1e-3), "matches": m, "count_ok": True}


def bench_c3(hj, torch, dev, steps, warmup) -> dict:
    """R = permutation of 1..2^24, S = 2^26 Zipf draws over R's keys (every S tuple
    matches once; at theta 1 the most frequent key holds ~5.8% of S)."""
    from paper_1307_1955_amd.gen import device as dgen
    out = {}
    for theta in (0.5, 1.0):
        t = dgen.config_c3(theta=theta, device=dev)
        n_s = t[2].numel()
        o_r = torch.empty(n_s, dtype=torch.int32, device=dev)
        o_s = torch.empty(n_s, dtype=torch.int32, device=dev)
        d = torch.zeros(1, dtype=torch.int64, device=dev)
        row = {}
        for name, q in (("phj", hj.params("phj", 2, (6, 6), one_pass=True)), ("shj", hj.params("shj", one_pass=True))):
            row[name] = timed_join(hj, torch, q, t, o_r, o_s, d, steps, warmup, n_s, dev)
        out["theta_%g" % theta] = row
        del t, o_r, o_s
        torch.cuda.empty_cache()
    return out


def bench_radix_sweep(hj, torch, t, out_r, out_s, d_count, want, dev) -> dict:
    """The 16M x 16M workload over radix bits 6-14 in one pass (up to 13, the
    per-pass limit) and in two passes (the split of HJ_AUTO), each with one- and
    two-pass output: time per join, every count against the closed form, and
    the best GB/s each phase reached over the sweep (per-kernel HIP events)."""
    n_r, n_s = t[0].numel(), t[2].numel()
    configs = [(1, (b,)) for b in range(6, 14)] + [(2, ((b + 1) // 2, b // 2)) for b in range(6, 15)]
    rows, best = [], {}
    for passes, bb in configs:
        for one in (True, False):
            q = hj.params("phj", passes, bb, one_pass=one)
            row = {"passes": passes, "bits": list(bb), "one_pass": one,
                   "tile": hj.hj_resolve_params(q, n_r, n_s).tile,
                   **timed_join(hj, torch, q, t, out_r, out_s, d_count, 5, 2, want, dev)}
            ws = hj.workspace(q, n_r, n_s, dev)
            for name, r in summarize(kernel_times(hj, q, t, out_r, out_s, ws, d_count, 1), 1, n_r, n_s,
                                     want).items():
                if "gbs" in r and r["gbs"] > best.get(name, {}).get("gbs", 0.0):
                    best[name] = {"gbs": r["gbs"], "frac_of_peak": round(r["gbs"] / HBM_PEAK_GBS, 4),
                                  "passes": passes, "bits": list(bb), "one_pass": one}
            del ws
            rows.append(row)
            print("bench: radix sweep %s" % row, file=sys.stderr, flush=True)
    fastest = min(rows, key=lambda r: r["ms"])
    return {"configs": rows, "best_per_phase_gbs": best,
            "fastest": {k: fastest[k] for k in ("passes", "bits", "one_pass", "ms", "tuples_per_s")}}


def bench_sweeps(hj, torch, dev, steps, warmup) -> dict:
    """Build-size sweep (|R| = 2^16..2^24, |S| = 2^24 uniform over 1..2|R|),
    selectivity sweep (16M x 16M, S uniform over 1..|R|/f for a match fraction f)
    and the low/high-skew sets (10% / 25% of R on one key) at three build sizes;
    every count against the closed form."""
    from paper_1307_1955_amd.gen import device as dgen
    n_s = 1 << 24
    o_r = torch.empty(n_s, dtype=torch.int32, device=dev)
    o_s = torch.empty(n_s, dtype=torch.int32, device=dev)
    d = torch.zeros(1, dtype=torch.int64, device=dev)

    def run(t):
        row = {}
        n_r = t[0].numel()
        want = device_count(torch, t[0], t[2])
        for name, q in (("phj_auto", hj.params("auto", one_pass=True)), ("shj", hj.params("shj", one_pass=True))):
            row[name] = timed_join(hj, torch, q, t, o_r, o_s, d, steps, warmup, want, dev)
            if name == "phj_auto":
                row[name]["params"] = repr(hj.hj_resolve_params(q, n_r, n_s))
        return row

    build = []
    for lg in (16, 18, 20, 22, 24):
        n_r = 1 << lg
        t = dgen.unique_uniform(7, n_r, n_s, 2 * n_r, dev)
        build.append({"n_r": n_r, "n_s": n_s, **run(t)})
        print("bench: build-size sweep %s" % build[-1], file=sys.stderr, flush=True)
        del t
    sel = []
    for f in (0.125, 0.5, 1.0):
        n_r = 1 << 24
        t = dgen.unique_uniform(8, n_r, n_s, int(n_r / f), dev)
        sel.append({"match_fraction": f, **run(t)})
        print("bench: selectivity sweep %s" % sel[-1], file=sys.stderr, flush=True)
        del t
    del o_r, o_s
    torch.cuda.empty_cache()
    return {"build_size": build, "selectivity": sel, "skew": bench_skew(hj, torch, dev, steps, warmup, (16, 20))}


def bench_skew(hj, torch, dev, steps, warmup, log2_sizes=(24,)) -> list:
    """The skewed sets of Section 5.1: |S| = 2^24 uniform over 1..2|R|, a fraction
    s = 10% (low) or 25% (high) of R's rows on one key, PHJ (`HJ_AUTO`) and SHJ;
    counts against the closed form."""
    from paper_1307_1955_amd.gen import device as dgen
    n_s = 1 << 24
    o_r = torch.empty(n_s, dtype=torch.int32, device=dev)
    o_s = torch.empty(n_s, dtype=torch.int32, device=dev)
    d = torch.zeros(1, dtype=torch.int64, device=dev)
    rows = []
    for frac in (0.10, 0.25):
        for lg in log2_sizes:
            n_r = 1 << lg
            t = dgen.skewed_r(9, n_r, n_s, 2 * n_r, frac, dev)
            want = device_count(torch, t[0], t[2])
            row = {"skew": frac, "n_r": n_r, "n_s": n_s}
            for name, q in (("phj_auto", hj.params("auto", one_pass=True)), ("shj", hj.params("shj", one_pass=True))):
                row[name] = timed_join(hj, torch, q, t, o_r, o_s, d, steps, warmup, want, dev)
            rows.append(row)
            print("bench: skew set %s" % row, file=sys.stderr, flush=True)
            del t
    del o_r, o_s
    torch.cuda.empty_cache()
    return rows


PROFILE = os.path.join(ROOT, "profiles", "phj_16m_x_16m_hbm.json")
KERNEL_OF_PHASE = {"part_hist": "k_part_hist", "part_scatter": "k_part_scatter", "join_count": "k_join_count",
                   "join_write": "k_join_write<false", "join_write_1pass": "k_join_write<true",
                   "shj_build": "k_shj_build", "shj_count": "k_shj_count", "shj_write": "k_shj_write<false",
                   "shj_write_1pass": "k_shj_write<true"}
# What the rocprofv3 counters FETCH_SIZE and WRITE_SIZE count: bytes between the
# L2 caches and the memory fabric, so lines served by the 256 MB Infinity Cache
# (MALL) count too; HBM itself may have moved fewer.
TRAFFIC_KIND = "beyond-L2 bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated; includes Infinity Cache hits)"


def counter_traffic(phase: str):
    """HBM bytes per launch of `phase` from the committed rocprofv3 counters, or
    None when there are none or the kernel sources changed since they were taken."""
    try:
        from paper_1307_1955_amd import profsum
        with open(PROFILE) as f:
            rec = json.load(f)
        if rec.get("sources_sha256") != profsum.sources_hash():
            return None
        want = KERNEL_OF_PHASE.get(phase)
        for r in rec["kernels"]:
            if want and r["kernel"].startswith(want) and r["hbm_read_mb"] is not None:
                return round((r["hbm_read_mb"] + r["hbm_write_mb"]) * 1e6, 0)
    except (OSError, ValueError, KeyError):
        return None
    return None


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the join runs on a single MI355X; multi-GPU sharding is a design "
              "note only (--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        x = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "launches": 3}), flush=True)
        return

    import paper_1307_1955_amd.hj as hj
    from paper_1307_1955_amd.gen import device as dgen

    dev = torch.device("cuda:0")
    n = args.n
    bits = tuple(int(b) for b in args.bits.split(","))
    one_pass = not args.two_pass
    p = hj.params("phj", args.passes, bits, hash=args.hash, tile=args.tile, one_pass=one_pass)
    rp = hj.hj_resolve_params(p, n, n)  # tile and LDS table capacity as the library chooses them
    print("bench: generating 16M x 16M inputs on the device", file=sys.stderr, flush=True)
    t = dgen.config_c2(n=n, device=dev)
    n_r, n_s = n, n
    out_r = torch.empty(n_s, dtype=torch.int32, device=dev)
    out_s = torch.empty(n_s, dtype=torch.int32, device=dev)
    d_count = torch.zeros(1, dtype=torch.int64, device=dev)

    print("bench: PHJ %r, %d warmup + %d timed steps" % (p, args.warmup, args.steps), file=sys.stderr, flush=True)
    head = measure_phj(hj, torch, p, t, out_r, out_s, d_count, n_r, n_s, args.steps, args.warmup, args.passes,
                       one_pass)
    phases = head["kernels"]
    m = head["matches"]
    want = int((t[2] <= n).sum())  # R keys are 1..|R|: every S key <= |R| matches once
    if m != want:
        raise AssertionError("PHJ produced %d pairs, the closed form says %d" % (m, want))
    # dominant kernel: most time per join among kernels with an algorithmic byte count
    dom = max((k for k in phases if "gbs" in phases[k]), key=lambda k: phases[k]["ms_per_join"])
    dom_bytes = algorithmic_bytes(dom, n_r, n_s, m)
    dom_ms = phases[dom]["avg_launch_ms"]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    result = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded, generated in HBM)",
        "config": {
            "workload": "PHJ 16M x 16M: |R| = |S| = %d int32 (key, rid); R keys a permutation of 1..|R|, "
                        "S keys uniform over 1..2|R| (~50%% match)" % n,
            "algo": "phj", "passes": args.passes, "bits": list(bits), "hash": args.hash,
            "tile": rp.tile, "lds_cap": rp.lds_cap, "output": "one-pass (block reservation)" if one_pass else
            "two-pass (count, scan, write)", "matches": m, "count_matches_closed_form": True,
        },
        "roofline": {
            "bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(dom),
            "traffic_kind": TRAFFIC_KIND, "bytes_per_launch": dom_bytes, "avg_launch_ms": dom_ms,
        },
        "path_gbs": head["path_gbs"],
        "path_frac": head["path_frac"],
        "clock_ramp_ms": head["clock_ramp_ms"],  # untimed joins before the warm-up steps (steady clocks)
        "kernels": phases,
    }
    if not args.no_extras:
        print("bench: build once, probe (split join)", file=sys.stderr, flush=True)
        result["build_probe"] = bench_build_probe(hj, torch, p, t, out_r, out_s, d_count, args.steps, args.warmup)
    # the other output materialisation on the same inputs (both give the same multiset)
    q = hj.params("phj", args.passes, bits, hash=args.hash, tile=args.tile, one_pass=not one_pass)
    alt = measure_phj(hj, torch, q, t, out_r, out_s, d_count, n_r, n_s, args.steps, args.warmup, args.passes,
                      not one_pass)
    result["two_pass_output" if one_pass else "one_pass_output"] = alt
    if not args.no_shj:
        for shj_one in (True, False):
            ps = hj.params("shj", one_pass=shj_one)
            ws_s = hj.workspace(ps, n_r, n_s, dev)
            print("bench: SHJ (%s output)" % ("one-pass" if shj_one else "two-pass"), file=sys.stderr, flush=True)
            ms_s = time_steps(lambda: hj.hj_join(ps, *t, out_r, out_s, ws_s, d_count), args.steps, args.warmup,
                              torch)
            m_s = int(d_count.item())
            if m_s != want:
                raise AssertionError("SHJ produced %d pairs, the closed form says %d" % (m_s, want))
            acc_s = kernel_times(hj, ps, t, out_r, out_s, ws_s, d_count, 5)
            ks = summarize(acc_s, 5, n_r, n_s, m_s)
            for name, row in ks.items():
                # one table lookup chain per R tuple inserted or S tuple probed
                units = {"shj_build": n_r, "shj_count": n_s, "shj_write": n_s, "shj_write_1pass": n_s}.get(name)
                if units:
                    row["random_accesses_per_s"] = units / (row["avg_launch_ms"] * 1e-3)
                    tb = counter_traffic(name)
                    row["counter_bytes_per_tuple"] = None if tb is None else round(tb / units, 1)
            result["shj" if shj_one else "shj_two_pass_output"] = {
                "value": (n_r + n_s) / (ms_s * 1e-3), "unit": "tuples/s", "ms_per_step": ms_s, "matches": m_s,
                "count_matches_closed_form": True, "kernels": ks,
                "counter_bytes_kind": TRAFFIC_KIND.replace(" per launch", "")}
            del ws_s
    if not args.no_sweeps and not args.no_extras:
        print("bench: radix sweep of the 16M x 16M workload", file=sys.stderr, flush=True)
        result["radix_sweep"] = bench_radix_sweep(hj, torch, t, out_r, out_s, d_count, m, dev)
    del out_r, out_s, t
    torch.cuda.empty_cache()
    if not args.no_c3 and not args.no_extras:
        print("bench: Zipf-skewed 16M x 64M (C3)", file=sys.stderr, flush=True)
        result["c3"] = bench_c3(hj, torch, dev, min(args.steps, 10), min(args.warmup, 3))
        print("bench: skewed R (10% / 25% on one key), 16M x 16M", file=sys.stderr, flush=True)
        result["skew"] = bench_skew(hj, torch, dev, min(args.steps, 10), min(args.warmup, 3))
    if not args.no_sweeps and not args.no_extras:
        result["sweeps"] = bench_sweeps(hj, torch, dev, min(args.steps, 10), min(args.warmup, 3))
    if args.batch_jobs:
        from paper_1307_1955_amd import tune, workloads
        print("bench: building the batched workload (%d jobs) in HBM" % args.batch_jobs, file=sys.stderr, flush=True)
        wl = workloads.batch_workload(njobs=args.batch_jobs)
        table = tune.load_table()
        params = workloads.tuned_params(wl.specs, table)
        result["batched"] = bench_batched(args, torch, hj, wl, params, table)
        if args.serve_requests:
            rate = result["batched"]["value"]
            result["served"] = bench_served(args, torch, hj, wl, params, [0.5 * rate, 0.8 * rate])
        del wl
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(n)
        print("bench: CPU oracle baseline, all host threads", file=sys.stderr, flush=True)
        result["cpu_baseline_all_cores"] = cpu_baseline_all_cores(n)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
