"""Device-resident synthetic workloads for the batched and served forms.

The batched workload: `njobs` independent joins, |R_j| log-uniform in
[r_min, r_max], |S_j| = |R_j| * U{1..max_factor}, R keys a permutation of
1..|R_j|, S keys uniform over 1..ceil(|R_j| / m_j) with m_j ~ U[0.25, 1]
(a 25-100% match rate); rid = row index.  Keys of all jobs live in two flat
HBM buffers; every job's rid columns are prefixes of one shared row-index
buffer (inputs are read-only, so sharing changes no result and no traffic).
Output buffers are sized to each job's exact pair count (every S key <= |R_j|
matches exactly one R tuple), computed on the device with plain PyTorch.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import gen
from .gen import device as dgen


@dataclass
class BatchWorkload:
    specs: list
    jobs: list            # per job: [r_key, r_rid, s_key, s_rid, out_r, out_s]
    d_counts: torch.Tensor
    expected: list        # exact pair count per job
    tuples: int           # sum of |R_j| + |S_j|
    pairs: int            # sum of expected counts
    input_bytes: int
    output_bytes: int


def batch_workload(seed: int = 4, njobs: int = 4096, r_min: int = gen.JOB_R_MIN, r_max: int = gen.JOB_R_MAX,
                   max_factor: int = 16, device="cuda") -> BatchWorkload:
    specs = gen.batch_specs(seed, njobs, r_min, r_max, max_factor)
    tot_r = sum(s.n_r for s in specs)
    tot_s = sum(s.n_s for s in specs)
    max_n = max([1] + [max(s.n_r, s.n_s) for s in specs])
    rkeys = torch.empty(max(1, tot_r), dtype=torch.int32, device=device)
    skeys = torch.empty(max(1, tot_s), dtype=torch.int32, device=device)
    rows = dgen.rows(max_n, device)
    views = []
    ro = so = 0
    cnt = torch.empty(len(specs), dtype=torch.int64, device=device)
    for j, sp in enumerate(specs):
        rk = rkeys[ro: ro + sp.n_r]
        sk = skeys[so: so + sp.n_s]
        dgen.perm_keys(sp.seed, sp.r_stream, sp.n_r, device, out=rk)
        dgen.uniform_keys(sp.seed, sp.s_stream, sp.n_s, sp.s_domain, device, out=sk)
        cnt[j] = (sk <= sp.n_r).sum()
        views.append((rk, rows[: sp.n_r], sk, rows[: sp.n_s]))
        ro += sp.n_r
        so += sp.n_s
    expected = cnt.cpu().tolist()
    total_pairs = int(sum(expected))
    out_r = torch.empty(max(1, total_pairs), dtype=torch.int32, device=device)
    out_s = torch.empty(max(1, total_pairs), dtype=torch.int32, device=device)
    jobs = []
    oo = 0
    for (rk, rr, sk, sr), e in zip(views, expected):
        jobs.append([rk, rr, sk, sr, out_r[oo: oo + e], out_s[oo: oo + e]])
        oo += e
    d_counts = torch.zeros(len(specs), dtype=torch.int64, device=device)
    return BatchWorkload(specs, jobs, d_counts, expected, tot_r + tot_s, total_pairs,
                         8 * (tot_r + tot_s), 8 * total_pairs)


def tuned_params(specs, table=None):
    """Per-job hj_params: the cost model's choice (HJ_AUTO, one-pass output), or
    a tuned table's bucket when a table is given."""
    from . import tune
    return [tune.choose(sp.n_r, sp.n_s, table).params() for sp in specs]


def verify_device(wl: BatchWorkload, counts: torch.Tensor | None = None, jobs=None) -> list:
    """Checks job outputs on the device against what the workload fixes, with
    plain PyTorch ops: the count equals the closed form (every S key <= |R_j|
    matches exactly one R tuple), every pair's R row and S row carry equal keys
    (rid = row index), and no S row appears twice.  Together these say that
    each matching S row appears exactly once, with the one R row of its key.
    counts: the counts to check (default wl.d_counts), one per job; jobs: the
    job indices (default all).  Returns the failing jobs as (job, reason)."""
    counts = wl.d_counts if counts is None else counts
    got = counts.cpu().tolist()
    bad = []
    for j in (range(len(wl.jobs)) if jobs is None else jobs):
        rk, _, sk, _, o_r, o_s = wl.jobs[j]
        c = wl.expected[j]
        if got[j] != c:
            bad.append((j, "count %d, closed form %d" % (got[j], c)))
            continue
        if c == 0:
            continue
        a, b = o_r[:c], o_s[:c]
        # rows in range before any gather
        lo_a, hi_a = torch.aminmax(a)
        lo_b, hi_b = torch.aminmax(b)
        if int(lo_a) < 0 or int(hi_a) >= rk.numel() or int(lo_b) < 0 or int(hi_b) >= sk.numel():
            bad.append((j, "row out of range"))
            continue
        if not torch.equal(rk.index_select(0, a), sk.index_select(0, b)):
            bad.append((j, "a pair joins unequal keys"))
            continue
        seen = torch.zeros(sk.numel(), dtype=torch.int32, device=sk.device)
        seen.index_fill_(0, b.long(), 1)
        if int(seen.sum()) != c:
            bad.append((j, "an S row appears twice"))
    return bad
