// Device-side helpers shared by the join kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hj_internal.h"

namespace hj {

constexpr int kWave = 64;
constexpr uint64_t kEmptySlot = ~0ull;  // empty slot of the HBM hash tables

// MurmurHash 2.0 (32-bit) of one 4-byte block, from Appleby's public description.
__device__ __forceinline__ uint32_t murmur2(uint32_t k) {
    const uint32_t m = 0x5bd1e995u;
    uint32_t h = 0x9747b28cu ^ 4u;
    k *= m;
    k ^= k >> 24;
    k *= m;
    h *= m;
    h ^= k;
    h ^= h >> 13;
    h *= m;
    h ^= h >> 15;
    return h;
}

// The value whose low bits select the partition (hj_hash).
__device__ __forceinline__ uint32_t radix_hash(int32_t key, uint32_t kind) {
    return kind ? murmur2((uint32_t)key) : (uint32_t)key;
}

// Full-avalanche 32-bit mixer (the MurmurHash3 finaliser) used to place keys in
// hash tables; independent of the radix bits so a partition's table is uniform.
__device__ __forceinline__ uint32_t slot_hash(int32_t key) {
    uint32_t h = (uint32_t)key;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// ---- Open-addressing tables with per-key rid chains (SHJ and HBM partition tables).
// A slot holds (key, head): key in the low 32 bits, the head of the key's row
// chain in the high 32.  kLast in a head/next field marks the chain's last row,
// so a key seen once costs one slot and no chain read.  The empty slot is all
// ones: its row field 0x7FFFFFFF can never be a row (n < 2^31 rows).
constexpr uint32_t kLast = 0x80000000u;
constexpr uint32_t kNotFound = 0xFFFFFFFFu;

__device__ __forceinline__ uint64_t chain_slot(int32_t key, uint32_t head) {
    return ((uint64_t)head << 32) | (uint32_t)key;
}

constexpr uint64_t kClaimed = ~0ull;  // chain_claim: the row took an empty slot

// Finds key k's slot, probing from slot s with step(s).  A row whose key is
// new claims an empty slot with one compare-and-swap and is done (kClaimed);
// otherwise the key's slot is returned and the row still has to be pushed
// onto its chain (WavePush).
template <typename Step>
__device__ __forceinline__ uint64_t chain_claim(uint64_t* table, uint64_t s, int32_t k, uint32_t row, Step step) {
    while (true) {
        // Read first and CAS only a free slot (faster on MI355X than an
        // unconditional CAS: the read brings the line in, the CAS then hits it).
        uint64_t cur = __hip_atomic_load(&table[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == kEmptySlot) {
            cur = atomicCAS((unsigned long long*)&table[s], (unsigned long long)kEmptySlot,
                            (unsigned long long)chain_slot(k, row | kLast));
            if (cur == kEmptySlot) return kClaimed;
        }
        if ((uint32_t)cur == (uint32_t)k) return s;
        s = step(s);
    }
}

// Keys that a build workgroup pushed kHotRun or more times in one run (the
// heavy keys of a skewed R), recorded by the SHJ build and the PHJ HBM-table
// build so that their probes can hand such tuples over without walking their
// chains first.  rows[i] sums the rows of key[i]'s recorded runs: a lower
// bound of its chain length (shorter runs are not counted), so a probe may
// skip the walk only when that bound alone exceeds its walk limit.  n may exceed kHotKeys; the keys beyond are
// not recorded.  A key may hold two entries (two workgroups recording it at
// once); each entry's rows stay a lower bound.
constexpr uint32_t kHotKeys = 63;
constexpr uint32_t kHotRun = 16;
struct HotKeys {
    uint32_t n;
    int32_t key[kHotKeys];
    uint32_t rows[kHotKeys];
    uint32_t valid[kHotKeys];  // 1 once key[i] is written (read during the build)
};

__device__ __forceinline__ void record_hot(HotKeys* hot, int32_t key, uint32_t rows) {
    const uint32_t n = min(__hip_atomic_load(&hot->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), kHotKeys);
    for (uint32_t i = 0; i < n; ++i) {
        if (__hip_atomic_load(&hot->valid[i], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) && hot->key[i] == key) {
            atomicAdd(&hot->rows[i], rows);
            return;
        }
    }
    const uint32_t idx = atomicAdd(&hot->n, 1u);
    if (idx < kHotKeys) {
        hot->key[idx] = key;
        atomicAdd(&hot->rows[idx], rows);
        __hip_atomic_store(&hot->valid[idx], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The build's hot keys into LDS, for a probe that registers their tuples as
// heavy without walking (needs a barrier before the arrays are read).
__device__ __forceinline__ void load_hot(const HotKeys* hot, int32_t* hk, uint32_t* hr, uint32_t* nhk) {
    const uint32_t n = min(hot->n, kHotKeys);
    if (threadIdx.x == 0) *nhk = n;
    if (threadIdx.x < n) {
        hk[threadIdx.x] = hot->key[threadIdx.x];
        hr[threadIdx.x] = hot->rows[threadIdx.x];
    }
}

// Rows the build recorded for key q (0 if it is not among the hot keys).
__device__ __forceinline__ uint32_t hot_rows_of(int32_t q, const int32_t* hk, const uint32_t* hr, uint32_t nhk) {
    uint32_t rows = 0;
    for (uint32_t i = 0; i < nhk; ++i) rows = hk[i] == q ? max(rows, hr[i]) : rows;
    return rows;
}

// Pushes of duplicate keys by one wave.  A row is pushed in front of its key's
// chain by exchanging the slot's head, which cannot fail (a claimed slot keeps
// its key), so a heavy key costs no compare-and-swap retries.  Exchanges are
// saved twice over: lanes pushing onto the same slot in one call are linked
// among themselves (lowest lane in front), and the wave keeps that run as a
// pending chain (slot, key, head row, tail row) that later runs onto the same
// slot extend, with one exchange when the wave moves to another slot or
// flushes.  Links are written before the exchange publishes them; tables are
// read only after the build launch ends.  Every lane of the wave calls add()
// and flush() (wave-uniform control flow); the pending fields are uniform.
struct WavePush {
    uint64_t slot = kClaimed;
    int32_t key = 0;
    uint32_t head = 0, tail = 0;
    uint32_t len = 0;          // rows in the pending run
    HotKeys* hot_keys = nullptr;  // where runs of kHotRun or more rows record their key
    // The slot of the last key the wave pushed: a row with that key can skip
    // chain_claim (a claimed slot never moves), which keeps a heavy key's rows
    // off its slot's cache line.
    uint64_t hot_slot = kClaimed;
    int32_t hot_key = 0;

    __device__ __forceinline__ bool hot(int32_t k) const { return hot_slot != kClaimed && k == hot_key; }

    __device__ __forceinline__ void flush(uint64_t* table, uint32_t* next) {
        if (slot != kClaimed) {
            if (__lane_id() == 0) {
                const uint64_t prev =
                    atomicExch((unsigned long long*)&table[slot], (unsigned long long)chain_slot(key, head));
                next[tail] = (uint32_t)(prev >> 32);
                if (hot_keys && len >= kHotRun) record_hot(hot_keys, key, len);
            }
            slot = kClaimed;
        }
    }

    // The block's last step: the waves' pending runs onto one slot are joined
    // (lower wave in front) and go in with one exchange, so a heavy key costs
    // one exchange per block, not per wave.  Every thread of the block calls
    // it; `runs` is LDS for one run per wave, reusable when it returns.
    struct Run {
        uint64_t slot;
        int32_t key;
        uint32_t head, tail, len;
    };
    template <uint32_t kWaves>
    __device__ __forceinline__ void flush_block(uint64_t* table, uint32_t* next, Run* runs) {
        if (__lane_id() == 0) runs[threadIdx.x / kWave] = Run{slot, key, head, tail, len};
        slot = kClaimed;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (uint32_t i = 0; i < kWaves; ++i) {
                const Run a = runs[i];
                if (a.slot == kClaimed) continue;
                uint32_t t = a.tail, rows = a.len;
                for (uint32_t j = i + 1; j < kWaves; ++j) {
                    if (runs[j].slot == a.slot) {
                        next[t] = runs[j].head;
                        t = runs[j].tail;
                        rows += runs[j].len;
                        runs[j].slot = kClaimed;
                    }
                }
                const uint64_t prev =
                    atomicExch((unsigned long long*)&table[a.slot], (unsigned long long)chain_slot(a.key, a.head));
                next[t] = (uint32_t)(prev >> 32);
                if (hot_keys && rows >= kHotRun) record_hot(hot_keys, a.key, rows);
            }
        }
        __syncthreads();
    }

    // s: the lane's slot from chain_claim (kClaimed: nothing to push).
    __device__ __forceinline__ void add(uint64_t* table, uint32_t* next, uint64_t s, int32_t k, uint32_t row) {
        const uint32_t lane = __lane_id();
        uint64_t todo = __ballot(s != kClaimed);
        while (todo) {
            const int lead = __ffsll((unsigned long long)todo) - 1;
            const uint64_t ls = __shfl(s, lead);
            const int32_t lk = __shfl(k, lead);
            const uint64_t peers = __ballot(s == ls) & todo;
            todo &= ~peers;
            const int last = 63 - __clzll((long long)peers);
            const uint32_t first_row = __shfl(row, lead);
            const uint32_t last_row = __shfl(row, last);
            const uint64_t after = peers & ~((2ull << lane) - 1ull);
            const int succ = after ? __ffsll((unsigned long long)after) - 1 : (int)lane;
            const uint32_t succ_row = __shfl(row, succ);
            const uint32_t rows = (uint32_t)__popcll(peers);
            if (s == ls && after) next[row] = succ_row;
            if (ls == slot) {
                if ((int)lane == last) next[row] = head;  // the run goes in front of the pending chain
                head = first_row;
                len += rows;
            } else {
                flush(table, next);
                slot = hot_slot = ls;
                key = hot_key = lk;
                head = first_row;
                tail = last_row;
                len = rows;
            }
        }
    }
};

// Head field of key `k`'s chain, or kNotFound.
template <typename Step>
__device__ __forceinline__ uint32_t chain_find(const uint64_t* __restrict__ table, uint64_t s, int32_t k,
                                               Step step) {
    while (true) {
        const uint64_t e = table[s];
        if (e == kEmptySlot) return kNotFound;
        if ((uint32_t)e == (uint32_t)k) return (uint32_t)(e >> 32);
        s = step(s);
    }
}

// Length of the chain starting at head field `h` (h != kNotFound).
__device__ __forceinline__ uint32_t chain_len(const uint32_t* __restrict__ next, uint32_t h) {
    uint32_t c = 1;
    while (!(h & kLast)) {
        h = next[h];
        ++c;
    }
    return c;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Uses v here, on every path: a load or atomic that returns v is awaited at
// this point (an empty statement that only reads the register).  The
// compiler's waits on the vector-memory counter do not follow branches: a
// result that some path may still have in flight makes it wait on that
// counter again wherever the register is reused, and such a wait also waits
// for every store in flight, which serializes a store loop.
__device__ __forceinline__ void settle(uint32_t v) { __asm__ volatile("" ::"v"(v)); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const uint32_t l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Wave-wide inclusive prefix sum (64 lanes) through LDS-crossbar shuffles;
// used for 64-bit values.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const uint32_t l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T u = __shfl_up(v, d, kWave);
        if (l >= (uint32_t)d) v += u;
    }
    return v;
}

// 32-bit specialisation without LDS traffic: DPP row shifts (row_shr 1, 2, 4, 8)
// give inclusive sums inside each row of 16 lanes; the row totals (lanes 15,
// 31, 47) are then read into scalar registers and added to the later rows.
template <>
__device__ __forceinline__ uint32_t wave_incl_scan<uint32_t>(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
    const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
    const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)v, 47);
    const uint32_t l = lane_id();
    v += (l >= 16 ? r0 : 0u) + (l >= 32 ? r1 : 0u) + (l >= 48 ? r2 : 0u);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Exclusive prefix and total over the wave of per-lane pair counts `c`.
// Fast paths: every count 0 or 1 (unique build keys) -> ballot + popcount;
// small counts -> 32-bit DPP scan; otherwise a 64-bit shuffle scan.
__device__ __forceinline__ void wave_offsets(uint32_t c, uint64_t* excl, uint64_t* total) {
    if (__ballot(c > 1) == 0) {
        const uint64_t m = __ballot(c != 0);
        *excl = (uint64_t)__popcll(m & lanemask_lt());
        *total = (uint64_t)__popcll(m);
    } else if (__ballot(c >= (1u << 25)) == 0) {
        const uint32_t incl = wave_incl_scan(c);
        *excl = incl - c;
        *total = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
    } else {
        const uint64_t incl = wave_incl_scan((uint64_t)c);
        *excl = incl - c;
        *total = __shfl(incl, kWave - 1, kWave);
    }
}

// The same for counts below 2^25 (matches in an LDS table), in 32 bits.
__device__ __forceinline__ void wave_offsets32(uint32_t c, uint32_t* excl, uint32_t* total) {
    if (__ballot(c > 1) == 0) {
        const uint64_t m = __ballot(c != 0);
        *excl = (uint32_t)__popcll(m & lanemask_lt());
        *total = (uint32_t)__popcll(m);
    } else {
        const uint32_t incl = wave_incl_scan(c);
        *excl = incl - c;
        *total = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
    }
}

// Block-wide exclusive scan of one value per thread.  `wave_tot` is LDS scratch
// of at least blockDim/64 entries.  Returns the exclusive prefix; *total gets
// the block total.  Contains __syncthreads().
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* wave_tot, T* total) {
    const uint32_t l = lane_id();
    const uint32_t w = threadIdx.x / kWave;
    const uint32_t nw = blockDim.x / kWave;
    T incl = wave_incl_scan(v);
    if (l == kWave - 1) wave_tot[w] = incl;
    __syncthreads();
    T before = 0, tot = 0;
    for (uint32_t i = 0; i < nw; ++i) {
        T t = wave_tot[i];
        if (i < w) before += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return before + incl - v;
}

// In-place exclusive scan of an LDS array a[0..n) (n a multiple of 64) by the
// whole block.  Wave w scans a contiguous run of 64-element chunks with a
// running carry; `wave_tot` (LDS, >= blockDim/64 entries) then carries the
// wave totals across waves.  Returns the total.  Contains __syncthreads()
// (callers must sync before reading `a`).
__device__ __forceinline__ uint32_t lds_excl_scan(uint32_t* a, uint32_t n, uint32_t* wave_tot) {
    const uint32_t l = lane_id();
    const uint32_t w = threadIdx.x / kWave;
    const uint32_t nw = blockDim.x / kWave;
    const uint32_t nchunks = n / kWave;
    const uint32_t per = (nchunks + nw - 1) / nw;
    const uint32_t c0 = min(w * per, nchunks), c1 = min(c0 + per, nchunks);
    uint32_t carry = 0;
    for (uint32_t c = c0; c < c1; ++c) {
        const uint32_t v = a[c * kWave + l];
        const uint32_t incl = wave_incl_scan(v);
        a[c * kWave + l] = carry + incl - v;
        carry += (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
    }
    if (l == 0) wave_tot[w] = carry;
    __syncthreads();
    uint32_t off = 0, total = 0;
    for (uint32_t i = 0; i < nw; ++i) {
        const uint32_t t = wave_tot[i];
        off += i < w ? t : 0u;
        total += t;
    }
    if (off)
        for (uint32_t c = c0; c < c1; ++c) a[c * kWave + l] += off;
    return total;
}

// Scratch entries `lds_excl_scan` needs (one per wave of the largest block).
constexpr uint32_t kScanScratch = 16;

// Block index -> work index such that each of the 8 XCDs (which receive blocks
// round-robin) processes one contiguous range of work indices.  A bijection on
// [0, grid).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t grid) {
    constexpr uint32_t kXcd = 8;
    const uint32_t x = b % kXcd;
    const uint32_t i = b / kXcd;
    const uint32_t q = grid / kXcd, r = grid % kXcd;
    return x * q + (x < r ? x : r) + i;
}

// Work index of block b when only the first `live` blocks of the grid have
// work: the live blocks are spread over all XCDs (xcd_remap over [0, live));
// blocks past `live` keep their index and find no work.
__device__ __forceinline__ uint32_t live_remap(uint32_t b, uint32_t live) {
    return b < live ? xcd_remap(b, live) : b;
}

// ---- chained (decoupled look-back) scans across workgroups ----
// A status word: flag in the top two bits (0 unset, 1 aggregate, 2 inclusive),
// a value below 2^62.
constexpr uint64_t kStatusAggregate = 1ull << 62;
constexpr uint64_t kStatusInclusive = 2ull << 62;
constexpr uint64_t kStatusValue = (1ull << 62) - 1;

__device__ __forceinline__ uint64_t status_load(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void status_store(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by all 64 lanes of one wave of tile `tile` (tiles numbered by ticket):
// publishes the tile's sum `tot` (< 2^62) in st[tile], walks back over the
// predecessors' statuses 64 at a time, adding aggregates until it meets an
// inclusive prefix, publishes its own inclusive prefix and returns the sum of
// all predecessors.  A predecessor whose status stays unset for ctl.max_polls
// polls is taken as inclusive so the kernel still ends, and kErrLookback goes
// into the call's error word: the prefix is then wrong and the host reports
// the call as failed.
__device__ __forceinline__ uint64_t lookback_wave(uint64_t* st, uint32_t tile, uint64_t tot, const ScanCtl& ctl) {
    const uint32_t lane = lane_id();
    if (lane == 0 && !(ctl.stall && tile == 0))
        status_store(&st[tile], (tile == 0 ? kStatusInclusive : kStatusAggregate) | (tot & kStatusValue));
    uint64_t prefix = 0;
    int64_t j = (int64_t)tile - 1;
    while (j >= 0) {
        const int64_t idx = j - (int64_t)lane;  // lane 0 is the nearest predecessor
        uint64_t w = idx >= 0 ? status_load(&st[idx]) : kStatusInclusive;  // nothing before tile 0
        for (uint32_t polls = 0; __ballot((w >> 62) == 0) != 0 && polls < ctl.max_polls; ++polls) {
            if (polls > 8) __builtin_amdgcn_s_sleep(1);
            if ((w >> 62) == 0) w = status_load(&st[idx]);
        }
        if (__ballot((w >> 62) == 0) != 0 && lane == 0 && ctl.err)
            atomicOr((unsigned long long*)ctl.err, (unsigned long long)kErrLookback);
        const uint64_t incl = __ballot((w >> 62) != 1);  // inclusive (or, past the poll bound, unset)
        const uint32_t stop = incl ? (uint32_t)__ffsll((unsigned long long)incl) - 1 : kWave - 1;
        prefix += wave_sum(lane <= stop ? (w & kStatusValue) : 0ull);
        if (incl) break;
        j -= kWave;
    }
    if (lane == 0 && tile != 0) status_store(&st[tile], kStatusInclusive | ((prefix + tot) & kStatusValue));
    return prefix;
}

// Largest s in [0, n) with begin[s] <= v, for a nondecreasing begin[0..n].
template <typename T>
__device__ __forceinline__ uint32_t upper_index(const T* begin, uint32_t n, T v) {
    uint32_t lo = 0, hi = n;  // answer in [lo, hi)
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (begin[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace hj
