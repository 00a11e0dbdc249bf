"""Chain lengths the LDS-table probe walks, and what grouping probes by key-list
length could save (Section 3.3, "workload divergence").

The join kernel builds, per work item, a chained table over R_i in LDS: 2^h
chain heads, h = floor(log2(max(64, |R_i|))), a record per R tuple pushed on
the chain of its bucket (slot_hash(key) >> (32 - h)); a probe walks the whole
chain of its S key's bucket.  A wave probes 9 S keys per lane in lockstep, so
a wave's round takes as many steps as the longest chain among its 576 keys.
The paper groups tuples of similar key-list length so that a wave's lanes
finish together.  This computes, exactly (same hash, same layout), the walk
length of every S tuple of a 2-pass 6+6-bit PHJ (identity radix hash) over the
16M x 16M workload and over the 16M x 64M Zipf workloads, the steps of every
wave round as the kernel forms them, and the steps the same waves would take
if each work item's S keys were first sorted by walk length (the best grouping
can do).

``python -m paper_1307_1955_amd.chains`` prints one JSON row per workload.
"""
from __future__ import annotations

import numpy as np

from . import gen

KSU = 9              # S keys per lane of a probe round
WAVE = 64
WAVES = 8
ROUND = KSU * WAVE * WAVES   # 4608 S keys per round of a work item
CHUNK = 2 * ROUND            # S keys per work item


def slot_hash(k: np.ndarray) -> np.ndarray:
    """The table's 32-bit finaliser mix (the published MurmurHash3 finaliser)."""
    h = k.astype(np.uint32).astype(np.uint64)
    m = np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(16)
    h = (h * np.uint64(0x85EBCA6B)) & m
    h ^= h >> np.uint64(13)
    h = (h * np.uint64(0xC2B2AE35)) & m
    h ^= h >> np.uint64(16)
    return h


def walk_lengths(r_key: np.ndarray, s_key: np.ndarray, bits: int = 12):
    """Per S tuple: its partition and the length of the chain its probe walks."""
    mask = np.int64((1 << bits) - 1)
    rp = r_key.astype(np.int64) & mask
    sp = s_key.astype(np.int64) & mask
    r_len = np.bincount(rp, minlength=1 << bits)
    h = np.floor(np.log2(np.maximum(64, r_len))).astype(np.int64)  # heads per partition: 2^h
    # bucket of every R and S tuple inside its partition's table; global bucket id
    # = partition * 2^13 + bucket (h <= 13 for partitions up to 8192 tuples)
    rb = (slot_hash(r_key) >> (np.uint64(32) - h[rp].astype(np.uint64))).astype(np.int64)
    sb = (slot_hash(s_key) >> (np.uint64(32) - h[sp].astype(np.uint64))).astype(np.int64)
    chain = np.bincount(rp * (1 << 14) + rb, minlength=(1 << bits) << 14)
    return sp, chain[sp * (1 << 14) + sb]


def wave_steps(sp: np.ndarray, walk: np.ndarray, grouped: bool) -> tuple[int, int]:
    """Total lockstep steps over all wave rounds, and the walked records, when
    S is partitioned (stable order inside a partition) and each work item's S
    keys go to the waves as the kernel assigns them (grouped: sorted by walk
    length first)."""
    order = np.argsort(sp, kind="stable")
    sp, walk = sp[order], walk[order]
    starts = np.searchsorted(sp, np.arange(sp.max() + 2))
    total = 0
    for i in range(len(starts) - 1):
        w = walk[starts[i]: starts[i + 1]]
        for c0 in range(0, len(w), CHUNK):
            item = w[c0: c0 + CHUNK]
            for r0 in range(0, len(item), ROUND):
                rnd = item[r0: r0 + ROUND]
                if grouped:
                    rnd = np.sort(rnd)
                # wave v of the round takes keys [v * 576, (v + 1) * 576)
                for v in range(0, len(rnd), KSU * WAVE):
                    total += int(rnd[v: v + KSU * WAVE].max())
    return total, int(walk.sum())


def report(n: int = 1 << 24) -> list[dict]:
    rows = []
    r, s = gen.config_c2(n=n)
    cases = [("C2 16M x 16M (uniform S over 1..2^25)", r.key, s.key)]
    for theta in (0.5, 1.0):
        r3, s3 = gen.config_c3(theta=theta, n_r=n, n_s=4 * n)
        cases.append(("C3 16M x 64M, Zipf theta %.1f" % theta, r3.key, s3.key))
    for name, rk, sk in cases:
        sp, walk = walk_lengths(rk, sk)
        hist = np.bincount(walk, minlength=8)
        steps, work = wave_steps(sp, walk, grouped=False)
        steps_g, _ = wave_steps(sp, walk, grouped=True)
        rows.append({"workload": name, "mean_walk": float(walk.mean()),
                     "walk_share": {str(k): float(hist[k] / len(walk)) for k in range(min(len(hist), 8))},
                     "max_walk": int(walk.max()), "lane_utilisation": work / (steps * KSU * WAVE),
                     "steps": steps, "steps_grouped": steps_g, "grouping_saves": 1 - steps_g / steps})
    return rows


if __name__ == "__main__":
    import json
    for row in report():
        print(json.dumps(row))
