// Duplicate-heavy keys in the probe of an HBM chained table (the SHJ table and
// the partition-local tables of overflowing PHJ partitions).
//
// A key of R with a long row chain makes every S tuple that matches it walk
// the chain in one lane, serially, while the rest of its wave idles: the
// workload divergence of Section 3.3, at its worst under the skewed relations
// of Section 5.1 (s% of R on one key).  Such S tuples are "heavy": the lane
// registers the tuple in an LDS set instead of walking, and the workgroup
// then counts and writes the matches of every registered tuple together by
// scanning R's key column (coalesced, one rank per hit across the block).
// A scan costs about |R| / (8 * block) block steps, a walk c dependent loads,
// so a chain is heavy only when it is longer than both kHeavyChain and
// |R| / 256 (|R|: the rows the table holds).
#pragma once

#include "hj_device.h"

namespace hj {

constexpr uint32_t kHeavyChain = 64;
// Heavy tuples a workgroup takes per probe round; more fall back to walking.
constexpr uint32_t kMaxHeavy = 32;
// In a lane's count word: a registered heavy tuple, its index in the low bits
// (counts stay below 2^31).
constexpr uint32_t kHeavyBit = 0x80000000u;
constexpr uint32_t kHeavyMaxWaves = 16;  // largest block: 1024 threads
constexpr uint32_t kHeavyV = 8;          // R keys per thread per scan step (more costs the callers' registers)

__device__ __forceinline__ uint32_t heavy_limit(uint64_t r_len) {
    const uint64_t l = r_len >> 8;
    return l > kHeavyChain ? (uint32_t)min<uint64_t>(l, kHeavyBit - 1) : kHeavyChain;
}

__device__ __forceinline__ bool is_heavy(uint32_t c) { return (c & kHeavyBit) != 0; }

// The heavy tuples of one probe round (LDS).
struct HeavySet {
    uint32_t n;                  // tuples registered (may exceed kMaxHeavy: the rest walk)
    uint32_t queued;             // bit e: entry e was handed to other workgroups (count 0 here)
    int32_t key[kMaxHeavy];
    int32_t srid[kMaxHeavy];
    uint32_t rep[kMaxHeavy];     // first entry with the same key (its scan serves both)
    uint32_t cnt[kMaxHeavy];     // exact match counts
    uint64_t pos[kMaxHeavy];     // first output slot of each entry
    uint32_t wsum[kHeavyMaxWaves * kHeavyV];  // per-wave hit counts of one scan step
};

// Length of the chain at head field h, or lim + 1 if longer.
__device__ __forceinline__ uint32_t chain_len_bounded(const uint32_t* __restrict__ next, uint32_t h,
                                                      uint32_t lim) {
    uint32_t c = 1;
    while (!(h & kLast) && c <= lim) {
        h = next[h];
        ++c;
    }
    return c;
}

// Registers an S tuple whose chain starts at head field h in hs: returns
// kHeavyBit | entry, or the chain length when the set is full.
__device__ __forceinline__ uint32_t register_heavy(const uint32_t* __restrict__ next, uint32_t h, int32_t key,
                                                   int32_t srid, HeavySet* hs) {
    const uint32_t e = atomicAdd(&hs->n, 1u);
    if (e >= kMaxHeavy) return chain_len(next, h);
    hs->key[e] = key;
    hs->srid[e] = srid;
    return kHeavyBit | e;
}

// Count word of an S tuple whose chain starts at head field h: the chain
// length, or kHeavyBit | entry when the tuple is registered in hs.
__device__ __forceinline__ uint32_t heavy_or_len(const uint32_t* __restrict__ next, uint32_t h, uint32_t lim,
                                                 int32_t key, int32_t srid, HeavySet* hs) {
    const uint32_t c = chain_len_bounded(next, h, lim);
    if (c <= lim) return c;
    return register_heavy(next, h, key, srid, hs);
}

// Exact counts of the registered tuples: one scan of R's keys per distinct
// key, kV keys per thread per step (Len: an index type that holds r_len).
// kQueued: entries marked in hs->queued are skipped (count 0).  All threads of
// the block call it, after the registrations.
template <uint32_t kBlock, uint32_t kV, bool kQueued = false, typename Len>
__device__ __forceinline__ void heavy_counts(const int32_t* __restrict__ rk, Len r_len, HeavySet* hs) {
    constexpr uint32_t kWaves = kBlock / kWave;
    static_assert(kWaves <= kHeavyMaxWaves, "block too large for the heavy set");
    __syncthreads();  // registrations done
    const uint32_t ne = min(hs->n, kMaxHeavy);
    if (threadIdx.x < ne) {
        // queued entries are nobody's representative and have none
        const uint32_t queued = kQueued ? hs->queued : 0u;
        uint32_t r = (queued >> threadIdx.x) & 1u ? kMaxHeavy : threadIdx.x;
        for (uint32_t i = 0; i < threadIdx.x && r != kMaxHeavy; ++i) {
            if (!((queued >> i) & 1u) && hs->key[i] == hs->key[threadIdx.x]) {
                r = i;
                break;
            }
        }
        hs->rep[threadIdx.x] = r;
    }
    __syncthreads();
    const uint32_t w = threadIdx.x / kWave;
    for (uint32_t e = 0; e < ne; ++e) {
        if (hs->rep[e] != e) continue;  // uniform: LDS value
        const int32_t k = hs->key[e];
        uint32_t m = 0;
        Len j = threadIdx.x;
        for (; j + (Len)(kV - 1) * kBlock < r_len; j += (Len)kV * kBlock) {
            int32_t v[kV];
#pragma unroll
            for (uint32_t u = 0; u < kV; ++u) v[u] = rk[j + (Len)u * kBlock];
#pragma unroll
            for (uint32_t u = 0; u < kV; ++u) m += v[u] == k;
        }
        for (; j < r_len; j += kBlock) m += rk[j] == k;
        m = wave_sum(m);
        if (lane_id() == 0) hs->wsum[w] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0;
            for (uint32_t i = 0; i < kWaves; ++i) t += hs->wsum[i];
            hs->cnt[e] = t;
        }
        __syncthreads();
    }
    if (threadIdx.x < ne)
        hs->cnt[threadIdx.x] = !kQueued || hs->rep[threadIdx.x] < kMaxHeavy ? hs->cnt[hs->rep[threadIdx.x]] : 0u;
    __syncthreads();
}

// Writes the matches of every registered tuple into its slots hs->pos[e] ..
// hs->pos[e] + cnt - 1, in no particular order: one scan of R per distinct
// key, kV (<= 32) keys per thread per step; each wave takes slots for its hits
// of an element with one LDS atomic on the key's fill counter (no barrier in
// the scan), and consecutive hit lanes write consecutive slots.  Slots at or
// past `capacity` are not written.  All threads of the block call it, after
// the positions are set.  kRids: the step's rids are loaded with its keys
// (more registers, no dependent load per hit).
template <uint32_t kBlock, uint32_t kV, bool kRids = false, typename Len>
__device__ __forceinline__ void heavy_writes(const int32_t* __restrict__ rk, const int32_t* __restrict__ rr,
                                             Len r_len, HeavySet* hs, uint64_t capacity,
                                             int32_t* __restrict__ out_r, int32_t* __restrict__ out_s) {
    constexpr Len kStep = (Len)kV * kBlock;
    static_assert(kV <= 32 && kMaxHeavy <= sizeof(hs->wsum) / sizeof(uint32_t), "fill counters fit wsum");
    uint32_t* fill = hs->wsum;  // per representative entry
    __syncthreads();  // positions published
    const uint32_t ne = min(hs->n, kMaxHeavy);
    if (threadIdx.x < ne) fill[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t e = 0; e < ne; ++e) {
        if (hs->rep[e] != e) continue;
        const int32_t k = hs->key[e];
        for (Len j0 = 0; j0 < r_len; j0 += kStep) {
            // element u of the thread: row j0 + u * kBlock + threadIdx.x; rows
            // past the end read the last row (all loads issue together) and
            // do not count
            int32_t v[kV], rid[kRids ? kV : 1];
#pragma unroll
            for (uint32_t u = 0; u < kV; ++u) {
                const Len j = min(j0 + (Len)u * kBlock + threadIdx.x, r_len - 1);
                v[u] = rk[j];
                if (kRids) rid[u] = rr[j];
            }
            uint32_t bits = 0;
#pragma unroll
            for (uint32_t u = 0; u < kV; ++u)
                bits |= (j0 + (Len)u * kBlock + threadIdx.x < r_len && v[u] == k) ? 1u << u : 0u;
            for (uint32_t u = 0; u < kV; ++u) {
                const uint64_t m = __ballot((bits >> u) & 1u);
                if (m == 0) continue;  // uniform over the wave
                const int lead = __ffsll((unsigned long long)m) - 1;
                uint32_t base = 0;
                if ((int)lane_id() == lead) base = atomicAdd(&fill[e], (uint32_t)__popcll(m));
                base = __shfl(base, lead);
                if ((bits >> u) & 1u) {
                    const uint32_t rank = base + (uint32_t)__popcll(m & lanemask_lt());
                    const int32_t r = kRids ? rid[kRids ? u : 0] : rr[j0 + (Len)u * kBlock + threadIdx.x];
                    for (uint32_t e2 = e; e2 < ne; ++e2) {
                        if (hs->rep[e2] != e) continue;
                        const uint64_t at = hs->pos[e2] + rank;
                        if (at < capacity) {
                            out_r[at] = r;
                            out_s[at] = hs->srid[e2];
                        }
                    }
                }
            }
        }
    }
}

}  // namespace hj
