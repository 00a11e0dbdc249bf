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

// ---- Heavy S tuples shared by all workgroups (one-pass output) ----
// A workgroup hands the heavy tuples it registered to the queue (hand_off);
// every workgroup, once its own work is written, runs help_heavy: for each
// queued tuple it claims chunks of the tuple's R rows and writes its matches
// in them, each scan step reserving its slots on the running total (one-pass
// output has no fixed order, so no count is needed first).  A workgroup takes
// what is unclaimed and leaves; the workgroup that queued a tuple runs
// help_heavy too, so every chunk is written before the launch ends.  (The
// PHJ write adds helper workgroups that wait, bounded, for tuples that its
// last items may still queue: k_join_write.)

// Moves this block's registered heavy tuples to the queue while it has room
// (marked in hs->queued); a tuple that finds the queue full stays with the
// block's own scan of R (heavy_counts / heavy_writes).  All threads call it
// after the registrations.
__device__ __forceinline__ void hand_off(HeavyQueue* Q, HeavySet* hs, uint32_t r_off, uint32_t r_len) {
    __syncthreads();  // registrations done
    const uint32_t ne = min(hs->n, kMaxHeavy);
    if (threadIdx.x < ne) {
        const uint32_t idx = atomicAdd(&Q->n, 1u);
        if (idx < kHeavyJobs) {
            HeavyJob* J = &Q->job[idx];
            J->key = hs->key[threadIdx.x];
            J->srid = hs->srid[threadIdx.x];
            J->r_off = r_off;
            J->r_len = r_len;
            __hip_atomic_store(&J->valid, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            atomicOr(&hs->queued, 1u << threadIdx.x);
        }
    }
}

// A one-pass probe hands a tuple to the queue once its chain is longer than
// this: a lane walking further would hold its workgroup past the others
// (every step a dependent load), while a queued tuple costs one scan of R
// shared by the workgroups that are still running.
constexpr uint32_t kQueueWalk = 1024;

// Claims the next chunk of a phase for the block (thread 0 takes it, LDS
// broadcasts it).  sh: LDS scratch.
__device__ __forceinline__ uint32_t claim_chunk(uint32_t* counter, uint32_t* sh) {
    __syncthreads();  // sh free
    if (threadIdx.x == 0) sh[0] = atomicAdd(counter, 1u);
    __syncthreads();
    return sh[0];
}

// rk, rr: the columns the queued tuples' R rows index (job rows r_off ..
// r_off + r_len - 1).  sh: LDS scratch of 9 + kHeavyV * kBlock / 64 words.
template <uint32_t kBlock>
__device__ __forceinline__ void help_heavy(HeavyQueue* Q, const int32_t* __restrict__ rk,
                                           const int32_t* __restrict__ rr,
                                           unsigned long long* __restrict__ total, uint64_t capacity,
                                           int32_t* __restrict__ out_r, int32_t* __restrict__ out_s, uint32_t* sh) {
    constexpr uint32_t kWaves = kBlock / kWave;
    constexpr uint32_t kV = kHeavyV;
    static_assert(kHeavyJobs <= kBlock, "one thread per queued tuple looks for open work");
    uint32_t* cnt = sh + 8;  // kV * kWaves per-wave hit counts of a step
    const uint32_t w = threadIdx.x / kWave;
    __syncthreads();
    if (threadIdx.x == 0) sh[1] = min(__hip_atomic_load(&Q->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), kHeavyJobs);
    __syncthreads();
    const uint32_t nj = sh[1];
    if (nj == 0) return;
    while (true) {
        // the lowest queued tuple that still has unclaimed chunks (one thread looks at each)
        __syncthreads();
        if (threadIdx.x == 0) sh[6] = ~0u;
        __syncthreads();
        // relaxed: a hint only (an acquire would drop cache lines that the
        // running workgroups use at every look); the job taken is read after
        // an acquire of its flag below
        if (threadIdx.x < nj) {
            HeavyJob* J = &Q->job[threadIdx.x];
            if (__hip_atomic_load(&J->valid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &&
                __hip_atomic_load(&J->write_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                    (J->r_len + kHelpChunk - 1) / kHelpChunk)
                atomicMin(&sh[6], threadIdx.x);
        }
        __syncthreads();
        const uint32_t e = sh[6];
        if (e == ~0u) return;
        HeavyJob* J = &Q->job[e];
        __syncthreads();
        if (threadIdx.x == 0) {
            (void)__hip_atomic_load(&J->valid, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);  // orders the reads below
            sh[2] = (uint32_t)J->key;
            sh[3] = (uint32_t)J->srid;
            sh[7] = J->r_off;
            sh[8 + kV * kWaves] = J->r_len;
        }
        __syncthreads();
        const int32_t k = (int32_t)sh[2], srid = (int32_t)sh[3];
        const uint64_t r_off = sh[7], r_len = sh[8 + kV * kWaves];
        const uint32_t nchunks = (uint32_t)((r_len + kHelpChunk - 1) / kHelpChunk);
        while (true) {
            const uint32_t c = claim_chunk(&J->write_next, sh);
            if (c >= nchunks) break;
            const uint64_t lo = r_off + (uint64_t)c * kHelpChunk, hi = r_off + min((uint64_t)(c + 1) * kHelpChunk, r_len);
            for (uint64_t j0 = lo; j0 < hi; j0 += (uint64_t)kV * kBlock) {
                // element u of the thread: row j0 + u * kBlock + threadIdx.x; rows
                // past the chunk read its last row (all loads issue together) and
                // do not count
                int32_t v[kV];
#pragma unroll
                for (uint32_t u = 0; u < kV; ++u) v[u] = rk[min(j0 + (uint64_t)u * kBlock + threadIdx.x, hi - 1)];
                uint32_t bits = 0;
#pragma unroll
                for (uint32_t u = 0; u < kV; ++u)
                    bits |= (j0 + (uint64_t)u * kBlock + threadIdx.x < hi && v[u] == k) ? 1u << u : 0u;
#pragma unroll
                for (uint32_t u = 0; u < kV; ++u) {
                    const uint32_t nh = (uint32_t)__popcll(__ballot((bits >> u) & 1u));
                    if (lane_id() == 0) cnt[u * kWaves + w] = nh;
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    uint32_t t = 0;
                    for (uint32_t i = 0; i < kV * kWaves; ++i) t += cnt[i];
                    const unsigned long long b = t ? atomicAdd(total, (unsigned long long)t) : 0ull;
                    sh[4] = (uint32_t)b;
                    sh[5] = (uint32_t)(b >> 32);
                }
                __syncthreads();
                uint64_t base = (uint64_t)sh[4] | ((uint64_t)sh[5] << 32);
                for (uint32_t u = 0; u < kV; ++u) {
                    uint32_t before = 0, all = 0;
                    for (uint32_t i = 0; i < kWaves; ++i) {
                        const uint32_t t = cnt[u * kWaves + i];
                        before += i < w ? t : 0u;
                        all += t;
                    }
                    const uint64_t mk = __ballot((bits >> u) & 1u);
                    if ((bits >> u) & 1u) {
                        const uint64_t at = base + before + (uint32_t)__popcll(mk & lanemask_lt());
                        if (at < capacity) {
                            out_r[at] = rr[j0 + (uint64_t)u * kBlock + threadIdx.x];
                            out_s[at] = srid;
                        }
                    }
                    base += all;
                }
                __syncthreads();  // cnt and sh reused
            }
        }
    }
}

}  // namespace hj
