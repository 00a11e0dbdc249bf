// Join of the partition pairs of a PHJ ("apply SHJ on each partition pair",
// Algorithm 2; steps b1-b4 and p1-p4 of Algorithm 1 inside each pair).
//
// Work item = (partition pair i, chunk of up to kJoinChunk S tuples of S_i),
// probed kJoinSub tuples at a time.  One workgroup per item:
//  * |R_i| <= lds_cap: R_i becomes a chained table in LDS.  The paper's
//    bucket header + key list + rid list (Section 3.1) is laid out without an
//    allocator: one head word per bucket and one 64-bit record (key, link)
//    per R tuple at its own row; a tuple is pushed on its bucket's chain with
//    one LDS exchange (the latch of Section 3.3).  Probing walks the chain
//    (p3) and compares keys (p4); rids are read from HBM for matches only.
//  * |R_i| > lds_cap (few, large partitions: low radix bits, duplicate-heavy
//    R): the pair is joined through a partition-local open-addressing table
//    in HBM (2 |R_i| slots at twice R_i's offset, plus per-key row chains),
//    cleared by the pass-2 scatter (counted plans of up to 6 pass-2 bits) or
//    by a clear launch, and built by a build launch (compare-and-swap for a
//    new key, exchange pushes for duplicates); S tuples on very long chains
//    are counted and written by the whole workgroup (hj_heavy.h).
// Workgroups take items in groups of 16 consecutive ones per XCD
// (item_of_block), so one partition's items share that XCD's L2.
// Output: count pass -> per-wave counts -> scan -> write pass, which re-runs
// the same item and stores its pairs at the scanned offset, or one pass that
// reserves each round's pairs on a running total (Section 3.3's dynamic
// output allocation replaced by counting or by block reservation).
#include <algorithm>

#include "hj_device.h"
#include "hj_heavy.h"
#include "hj_internal.h"
#include "hj_side.h"

namespace hj {

namespace {

constexpr uint32_t kSubJ = kJoinSub / kJoinWaves;     // S tuples per wave of a probe round

__device__ __forceinline__ uint64_t region_slot(int32_t key, uint32_t H) {
    return ((uint64_t)slot_hash(key) * H) >> 32;
}

__global__ void __launch_bounds__(256) k_ovf_clear(const PartPair* __restrict__ pairs,
                                                  const uint32_t* __restrict__ ovf_begin,
                                                  const uint32_t* __restrict__ ovf_part, uint32_t P,
                                                  uint64_t* __restrict__ ovf_table) {
    const uint32_t nitems = ovf_begin[P];
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const uint32_t i = ovf_part[item];
        const uint32_t c = item - ovf_begin[i];
        const PartPair pp = pairs[i];
        uint64_t* region = ovf_table + 2ull * pp.r_off;
        const uint64_t H = 2ull * pp.r_len;
        const uint32_t chunk = ovf_chunk(pp.r_len);
        const uint64_t end = min(2ull * (c + 1) * chunk, H);
        for (uint64_t x = 2ull * c * chunk + threadIdx.x; x < end; x += blockDim.x) region[x] = kEmptySlot;
    }
}

struct RegionStep {
    uint32_t H;
    __device__ __forceinline__ uint64_t operator()(uint64_t s) const { return s + 1 == H ? 0 : s + 1; }
};

__global__ void __launch_bounds__(256) k_ovf_build(const PartPair* __restrict__ pairs,
                                                  const uint32_t* __restrict__ ovf_begin,
                                                  const uint32_t* __restrict__ ovf_part, uint32_t P,
                                                  const int32_t* __restrict__ rk,
                                                  uint64_t* __restrict__ ovf_table,
                                                  uint32_t* __restrict__ ovf_next, HotKeys* hot,
                                                  HeavyQueue* heavy) {
    constexpr uint32_t kWaves = 256 / kWave;
    __shared__ WavePush::Run runs[kWaves];
    const uint32_t nitems = ovf_begin[P];
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const uint32_t i = ovf_part[item];
        const uint32_t c = item - ovf_begin[i];
        const PartPair pp = pairs[i];
        uint64_t* region = ovf_table + 2ull * pp.r_off;
        uint32_t* next = ovf_next + pp.r_off;
        const RegionStep step{2u * pp.r_len};
        const uint32_t chunk = ovf_chunk(pp.r_len);
        const uint32_t end = min((c + 1) * chunk, pp.r_len);
        // a partition the one-pass write may queue tuples of: the write's helpers
        // wait until its work items are done
        if (heavy && c == 0 && threadIdx.x == 0 && pp.r_len > kHelpChunk) {
            atomicAdd(&heavy->items_expected, items_of(pp));
            heavy->wait = 1;
        }
        WavePush push;
        push.hot_keys = hot;
        for (uint32_t j0 = c * chunk; j0 < end; j0 += blockDim.x) {  // uniform trip count
            const uint32_t j = j0 + threadIdx.x;
            int32_t k = 0;
            uint64_t s = kClaimed;
            if (j < end) {
                k = rk[pp.r_off + j];
                s = push.hot(k) ? push.hot_slot : chain_claim(region, region_slot(k, step.H), k, j, step);
            }
            push.add(region, next, s, k, j);
        }
        push.flush_block<kWaves>(region, next, runs);
    }
}

constexpr uint32_t kSU = kSubJ / kWave;  // S tuples per lane of a probe round

static_assert(kRptLarge * kJoinBlock == kMaxLdsCap, "largest build covers kMaxLdsCap");

// Heads of the LDS table for n tuples: the largest power of two <= max(64, n)
// (chains of one tuple on average).
__device__ __forceinline__ uint32_t table_log2H(uint32_t n) {
    const uint32_t v = n < 64 ? 64u : n;
    return 31u - (uint32_t)__clz(v);
}

// R_i's keys of this thread, n <= RPT * kJoinBlock.  Plain loads: every S
// chunk (work item) of a partition reads R_i again.
template <uint32_t RPT>
__device__ __forceinline__ void load_r(const int32_t* __restrict__ rk, uint32_t n, int32_t* k) {
#pragma unroll
    for (uint32_t u = 0; u < RPT; ++u) {
        const uint32_t j = u * kJoinBlock + threadIdx.x;
        k[u] = j < n ? rk[j] : 0;
    }
}

// LDS table of a work item: one 64-bit record per R_i tuple at its row j --
// the key and the link to the next row of its bucket's chain -- and the chain
// heads (the paper's bucket header + key list of Section 3.1, with row
// indices in place of pointers).  The rid list stays in HBM: a match's rid is
// read from R_i's rid column at its row when the pair is written.  Layout:
//   heads[cap + 64] | spare[64] | rec[cap] (uint64: key | next << 32)
constexpr uint32_t kChainEnd = 0xFFFFFFFFu;
struct LdsView {
    uint32_t* heads;
    uint32_t* spare;
    uint64_t* rec;
};

__device__ __forceinline__ LdsView lds_view(uint32_t* lds, uint32_t cap) {
    LdsView v;
    v.heads = lds;
    v.spare = lds + cap + kWave;
    v.rec = (uint64_t*)(v.spare + kWave);  // 8-byte aligned: cap is a multiple of 64
    return v;
}

__device__ __forceinline__ int32_t rec_key(uint64_t r) { return (int32_t)(uint32_t)r; }
__device__ __forceinline__ uint32_t rec_next(uint64_t r) { return (uint32_t)(r >> 32); }

// Builds the table over the n <= RPT * kJoinBlock keys held in registers: b1-b2
// bucket of the key, b3-b4 the tuple is pushed on its bucket's chain with one
// LDS exchange (the latch of Section 3.3 is the exchange itself) and its record
// stored at its row.  Rounds past n are skipped as a whole (n is uniform over
// the block); inside a round, lanes past n exchange on a private spare word so
// the round's exchanges are issued without branches.
template <uint32_t RPT>
__device__ __forceinline__ void build_lds(const int32_t* k, uint32_t n, uint32_t log2H, const LdsView& v) {
    const uint32_t H = 1u << log2H;
    const uint32_t sh = 32 - log2H;
    for (uint32_t x = threadIdx.x; x < H; x += kJoinBlock) v.heads[x] = kChainEnd;
    __syncthreads();
#pragma unroll
    for (uint32_t u = 0; u < RPT; ++u) {
        if (u * kJoinBlock < n) {
            const uint32_t j = u * kJoinBlock + threadIdx.x;
            const uint32_t b = slot_hash(k[u]) >> sh;
            const uint32_t old = atomicExch(j < n ? &v.heads[b] : &v.spare[lane_id()], j);
            if (j < n) v.rec[j] = (uint64_t)(uint32_t)k[u] | ((uint64_t)old << 32);
        }
    }
    __syncthreads();
}

struct ItemLoc {
    uint32_t item;
    bool live;
    uint32_t r_off, r_len;
    uint32_t s_begin, s_n;
};

// The work item of this workgroup, one dependent load (the plan writes the
// records past the last item empty; an item has at least one S tuple).
// Workgroups go to the 8 XCDs round-robin; items are dealt to them in groups
// of kItemGroup consecutive items (the items of one partition share its table
// in the XCD's L2), so each XCD gets every 8th group, evenly however many
// items there are.  A bijection on a grid of a multiple of 8 kItemGroup.
__device__ __forceinline__ uint32_t item_of_block(uint32_t b) {
    const uint32_t x = b % 8, l = b / 8;
    return ((l / kItemGroup) * 8 + x) * kItemGroup + l % kItemGroup;
}

__device__ __forceinline__ ItemLoc locate_item(const ItemRec* __restrict__ item_rec) {
    ItemLoc L;
    L.item = item_of_block(blockIdx.x);
    const ItemRec r = item_rec[L.item];
    L.live = r.s_n != 0;
    L.r_off = r.r_off;
    L.r_len = r.r_len;
    L.s_begin = r.s_begin;
    L.s_n = r.s_n;
    return L;
}

// S keys (and rids) of this lane for the wave's range [wb, we) of the item
// (kNt: non-temporal loads, for large joins; see kNtMinTuples).
template <bool kRids, bool kNt = false>
__device__ __forceinline__ void load_s(const int32_t* __restrict__ skp, const int32_t* __restrict__ srp,
                                       uint32_t wb, uint32_t we, int32_t* q, int32_t* qr) {
#pragma unroll
    for (uint32_t u = 0; u < kSU; ++u) {
        const uint32_t j = wb + u * kWave + lane_id();
        q[u] = j < we ? (kNt ? __builtin_nontemporal_load(skp + j) : skp[j]) : 0;
        if (kRids) qr[u] = j < we ? (kNt ? __builtin_nontemporal_load(srp + j) : srp[j]) : 0;
    }
}

// p1-p4 for the lane's kSU S keys against the LDS table, without branches per
// key: the chain heads of all keys are read first, then the chains are walked
// in lockstep (each step reads the current record -- key and link -- for every
// key whose chain has not ended, at a clamped address), so each step keeps kSU
// LDS reads in flight and a wave runs only as many steps as its longest chain.
// cf[u] = matches | first << 16 (16-bit halves: cap < 2^16), first = row of
// the first match met (meaningful when there is one).
__device__ __forceinline__ void probe_lds(const LdsView& v, uint32_t log2H, const int32_t* q, uint32_t wb,
                                          uint32_t we, uint32_t* cf) {
    const uint32_t sh = 32 - log2H;
    uint32_t h[kSU];
#pragma unroll
    for (uint32_t u = 0; u < kSU; ++u) {
        const bool ok = wb + u * kWave + lane_id() < we;
        const uint32_t head = v.heads[slot_hash(q[u]) >> sh];
        h[u] = ok ? head : kChainEnd;
        cf[u] = 0;
    }
    while (true) {
        bool live = false;
#pragma unroll
        for (uint32_t u = 0; u < kSU; ++u) live |= h[u] != kChainEnd;
        if (__ballot(live) == 0) break;
        uint64_t rc[kSU];
#pragma unroll
        for (uint32_t u = 0; u < kSU; ++u) rc[u] = v.rec[h[u] != kChainEnd ? h[u] : 0u];
        __builtin_amdgcn_sched_barrier(0);  // keep the step's reads together, in flight at once
#pragma unroll
        for (uint32_t u = 0; u < kSU; ++u) {
            const bool on = h[u] != kChainEnd;
            const bool hit = on && rec_key(rc[u]) == q[u];
            const uint32_t first = (cf[u] & 0xFFFFu) == 0 ? h[u] << 16 : cf[u] & 0xFFFF0000u;
            cf[u] = hit ? first | ((cf[u] & 0xFFFFu) + 1u) : cf[u];
            h[u] = on ? rec_next(rc[u]) : kChainEnd;
        }
    }
}

// LDS of a work item whose R partition has an HBM table: the heavy set of a
// probe round and the hot keys the table's build recorded.
struct HbmLds {
    HeavySet hs;
    int32_t hk[kHotKeys];
    uint32_t hr[kHotKeys];
    uint32_t nhk;
};

// Matches of the lane's kSU S keys in the partition-local HBM table (H = 2
// r_len slots).  A key with a chain longer than lim is registered in `hs`
// (c[u] = kHeavyBit | its index) when there is room, else counted by walking;
// a hot key whose recorded rows alone exceed lim is registered without the
// walk.  hs->n must be zero and visible to the block before the call.
__device__ __forceinline__ void probe_hbm(const uint64_t* __restrict__ region, const uint32_t* __restrict__ next,
                                          uint32_t H, uint32_t lim, const int32_t* q, const int32_t* qr, uint32_t wb,
                                          uint32_t we, uint32_t* c, uint32_t* at, HbmLds* sh) {
    const RegionStep step{H};
#pragma unroll
    for (uint32_t u = 0; u < kSU; ++u) {
        c[u] = 0;
        at[u] = kNotFound;
        if (wb + u * kWave + lane_id() < we) {
            at[u] = chain_find(region, region_slot(q[u], H), q[u], step);
            if (at[u] != kNotFound) {
                const uint32_t hot = (at[u] & kLast) ? 0u : hot_rows_of(q[u], sh->hk, sh->hr, sh->nhk);
                c[u] = hot > lim ? register_heavy(next, at[u], q[u], qr ? qr[u] : 0, &sh->hs)
                                 : heavy_or_len(next, at[u], lim, q[u], qr ? qr[u] : 0, &sh->hs);
            }
        }
    }
}

// Writes the c >= 1 matches of `key` to o_r/o_s[p ...], slots below `room`
// only (o_r, o_s and room are the wave's output window: uniform base pointers
// and the capacity left there).  The first match is at row `first` and its
// rid, rid0, was fetched already; further matches follow the chain and read
// their rids from R_i's rid column `rrp`.
__device__ __forceinline__ void write_lds_matches(const LdsView& v, const int32_t* __restrict__ rrp, int32_t key,
                                                  int32_t rs, uint32_t first, int32_t rid0, uint32_t c, uint32_t p,
                                                  uint32_t room, int32_t* __restrict__ o_r,
                                                  int32_t* __restrict__ o_s) {
    if (p < room) {
        o_r[p] = rid0;
        o_s[p] = rs;
    }
    if (c == 1) return;
    ++p;
    for (uint32_t x = rec_next(v.rec[first]); x != kChainEnd; x = rec_next(v.rec[x])) {
        if (rec_key(v.rec[x]) == key) {
            if (p < room) {
                o_r[p] = rrp[x];
                o_s[p] = rs;
            }
            ++p;
        }
    }
}

// Wave-uniform copy of a 64-bit value held equal in every active lane.
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Block-wide output reservation for one probe round (the block allocator of
// Section 3.3 with a block sized to the round's pairs): one atomic add of the
// round's total on the running count.  `mine` = this lane's pairs.  Returns the
// first slot of this wave.  `again`: a previous round used `wtot` (uniform over
// the block).
// T: uint32_t for the LDS table (a round has at most kJoinSub x kMaxLdsCap
// pairs), uint64_t for the HBM table (duplicate-heavy R can exceed 2^32).
template <typename T>
__device__ __forceinline__ uint64_t block_reserve(T mine, unsigned long long* total, uint64_t* wtot,
                                                  bool again) {
    const uint32_t w = threadIdx.x / kWave;
    mine = wave_sum(mine);
    if (again) __syncthreads();  // every wave has read the previous round's offsets
    if (lane_id() == 0) wtot[w] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (uint32_t i = 0; i < kJoinWaves; ++i) t += wtot[i];
        wtot[kJoinWaves] = t ? atomicAdd(total, (unsigned long long)t) : 0ull;
    }
    __syncthreads();
    uint64_t pos0 = wtot[kJoinWaves];
    for (uint32_t i = 0; i < w; ++i) pos0 += wtot[i];
    return pos0;
}

__device__ __forceinline__ uint32_t lane_pairs_lds(const uint32_t* cf) {
    uint32_t m = 0;
#pragma unroll
    for (uint32_t u = 0; u < kSU; ++u) m += cf[u] & 0xFFFFu;
    return m;
}

// Stores the round's pairs of this wave from output slot pos0 on (wave-compacted
// by match counts); returns the slot after the wave's last pair.  LDS table.
// A round of a wave has fewer than 2^32 pairs (kSubJ keys x kMaxLdsCap
// matches), so slots are 32-bit offsets from the wave's uniform base.
__device__ __forceinline__ uint64_t write_round_lds(const LdsView& v, const int32_t* __restrict__ rrp,
                                                    const int32_t* q, const int32_t* qr, const uint32_t* cf,
                                                    const int32_t* rid0, uint64_t pos0, uint64_t capacity,
                                                    int32_t* __restrict__ out_r, int32_t* __restrict__ out_s) {
    pos0 = uniform64(pos0);
    const uint64_t left = capacity > pos0 ? capacity - pos0 : 0ull;
    const uint32_t room = left > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)left;
    int32_t* __restrict__ o_r = out_r + pos0;
    int32_t* __restrict__ o_s = out_s + pos0;
    uint32_t done = 0;  // pairs of the wave written so far
#pragma unroll
    for (uint32_t u = 0; u < kSU; ++u) {
        const uint32_t c = cf[u] & 0xFFFFu;
        uint32_t excl, wtotal;
        wave_offsets32(c, &excl, &wtotal);
        if (c) write_lds_matches(v, rrp, q[u], qr[u], cf[u] >> 16, rid0[u], c, done + excl, room, o_r, o_s);
        done += wtotal;
    }
    return pos0 + done;
}

// Rids of the first matches (issued right after the probe, so the loads are in
// flight during the output reservation).
__device__ __forceinline__ void fetch_first_rids(const int32_t* __restrict__ rrp, const uint32_t* cf, int32_t* rid0) {
#pragma unroll
    for (uint32_t u = 0; u < kSU; ++u) rid0[u] = (cf[u] & 0xFFFFu) ? rrp[cf[u] >> 16] : 0;
}

// The same for the partition-local HBM table: c[u] matches on the row chain
// that starts at at[u].
// Heavy entries (is_heavy(c[u])) take their count from hs and only publish
// their first slot in hs->pos; heavy_writes writes them.
__device__ __forceinline__ uint64_t write_round_hbm(const uint32_t* __restrict__ next,
                                                    const int32_t* __restrict__ rrp, const int32_t* qr,
                                                    const uint32_t* c, const uint32_t* at,
                                                    HeavySet* hs, uint64_t pos0, uint64_t capacity,
                                                    int32_t* __restrict__ out_r, int32_t* __restrict__ out_s) {
#pragma unroll
    for (uint32_t u = 0; u < kSU; ++u) {
        const bool heavy = is_heavy(c[u]);
        const uint32_t cu = heavy ? hs->cnt[c[u] & ~kHeavyBit] : c[u];
        uint64_t excl, wtotal;
        wave_offsets(cu, &excl, &wtotal);
        uint64_t pos = pos0 + excl;
        pos0 += wtotal;
        if (heavy) {
            hs->pos[c[u] & ~kHeavyBit] = pos;
        } else if (cu) {
            uint32_t h = at[u];
            while (true) {
                const uint32_t row = h & ~kLast;
                if (pos < capacity) {
                    out_r[pos] = rrp[row];
                    out_s[pos] = qr[u];
                }
                ++pos;
                if (h & kLast) break;
                h = next[row];
            }
        }
    }
    return pos0;
}

// Count pass over a partition whose R exceeds the LDS table: probes the
// partition-local HBM table and returns this lane's pair count.  hs takes the
// LDS the table would have used.  Inlined: a call would give the kernel a
// stack, and the LDS path measured a few percent slower with one.
__device__ __forceinline__ uint64_t join_count_hbm(const ItemLoc L, uint32_t w, const int32_t* __restrict__ rk,
                                                   const int32_t* __restrict__ skp,
                                                   const uint64_t* __restrict__ ovf_table,
                                                   const uint32_t* __restrict__ ovf_next, const HotKeys* hot,
                                                   HbmLds* sh) {
    HeavySet* hs = &sh->hs;
    uint64_t cnt = 0;
    int32_t q[kSU];
    load_hot(hot, sh->hk, sh->hr, &sh->nhk);  // read after the round's barrier
    for (uint32_t sb = 0; sb < L.s_n; sb += kJoinSub) {
        const uint32_t wb = sb + w * kSubJ, we = min(wb + kSubJ, L.s_n);
        load_s<false>(skp, nullptr, wb, we, q, nullptr);
        if (threadIdx.x == 0) hs->n = 0;
        __syncthreads();
        uint32_t c[kSU], at[kSU];
        probe_hbm(ovf_table + 2ull * L.r_off, ovf_next + L.r_off, 2u * L.r_len, heavy_limit(L.r_len), q, nullptr, wb,
                  we, c, at, sh);
        heavy_counts<kJoinBlock, kHeavyV>(rk + L.r_off, L.r_len, hs);
#pragma unroll
        for (uint32_t u = 0; u < kSU; ++u) cnt += is_heavy(c[u]) ? hs->cnt[c[u] & ~kHeavyBit] : c[u];
        __syncthreads();  // the set is reused by the next round
    }
    return cnt;
}

template <uint32_t RPT, bool kNt>
__global__ void __launch_bounds__(kJoinBlock) k_join_count(const PartPair* __restrict__ pairs,
                                                          const uint32_t* __restrict__ item_begin,
                                                          const ItemRec* __restrict__ item_rec,
                                                          uint32_t P, const int32_t* __restrict__ rk,
                                                          const int32_t* __restrict__ sk, uint32_t lds_cap,
                                                          const uint64_t* __restrict__ ovf_table,
                                                          const uint32_t* __restrict__ ovf_next,
                                                          const HotKeys* __restrict__ hot,
                                                          uint64_t* __restrict__ wave_cnt) {
    extern __shared__ uint32_t lds[];
    const uint32_t w = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const ItemLoc L = locate_item(item_rec);
    if (!L.live) {
        if (lane == 0) wave_cnt[(uint64_t)L.item * kJoinWaves + w] = 0;
        return;
    }
    const int32_t* __restrict__ skp = sk + L.s_begin;
    uint64_t cnt = 0;
    int32_t q[kSU];
    if (L.r_len <= lds_cap) {
        int32_t k[RPT];
        load_r<RPT>(rk + L.r_off, L.r_len, k);
        load_s<false, kNt>(skp, nullptr, w * kSubJ, min(w * kSubJ + kSubJ, L.s_n), q, nullptr);
        const LdsView v = lds_view(lds, lds_cap);
        const uint32_t log2H = table_log2H(L.r_len);
        build_lds<RPT>(k, L.r_len, log2H, v);
        for (uint32_t sb = 0; sb < L.s_n; sb += kJoinSub) {
            const uint32_t wb = sb + w * kSubJ, we = min(wb + kSubJ, L.s_n);
            if (sb) load_s<false, kNt>(skp, nullptr, wb, we, q, nullptr);
            uint32_t cf[kSU];
            probe_lds(v, log2H, q, wb, we, cf);
            cnt += lane_pairs_lds(cf);
        }
    } else {
        cnt = join_count_hbm(L, w, rk, skp, ovf_table, ovf_next, hot, reinterpret_cast<HbmLds*>(lds));
    }
    cnt = wave_sum(cnt);
    if (lane == 0) wave_cnt[(uint64_t)L.item * kJoinWaves + w] = cnt;
}

// Write pass over a partition whose R exceeds the LDS table (see
// join_count_hbm).  One-pass output with `heavy`: a heavy S tuple of a
// partition that spans more than one kHelpChunk-row chunk is registered after
// a walk of at most kQueueWalk rows (none for a recorded hot key) and handed
// to the device-wide queue, whose chunks every workgroup of the launch helps
// write (help_heavy); tuples the queue has no room for stay with this
// workgroup's own scans.
template <bool kOnePass>
__device__ __forceinline__ void join_write_hbm(
    const ItemLoc L, uint32_t w, const int32_t* __restrict__ rk, const int32_t* __restrict__ rrp,
    const int32_t* __restrict__ skp, const int32_t* __restrict__ srp, const uint64_t* __restrict__ ovf_table,
    const uint32_t* __restrict__ ovf_next, const HotKeys* hot, uint64_t base, unsigned long long* __restrict__ total,
    uint64_t* wtot, int32_t* __restrict__ out_r, int32_t* __restrict__ out_s, uint64_t capacity, HbmLds* sh,
    HeavyQueue* heavy) {
    HeavySet* hs = &sh->hs;
    const uint64_t* __restrict__ region = ovf_table + 2ull * L.r_off;
    const uint32_t* __restrict__ next = ovf_next + L.r_off;
    const bool queue = kOnePass && heavy && L.r_len > kHelpChunk;  // uniform
    const uint32_t lim = queue ? min(heavy_limit(L.r_len), kQueueWalk) : heavy_limit(L.r_len);
    int32_t q[kSU], qr[kSU];
    load_hot(hot, sh->hk, sh->hr, &sh->nhk);  // read after the round's barrier
    for (uint32_t sb = 0; sb < L.s_n; sb += kJoinSub) {
        const uint32_t wb = sb + w * kSubJ, we = min(wb + kSubJ, L.s_n);
        load_s<true>(skp, srp, wb, we, q, qr);
        if (threadIdx.x == 0) hs->n = hs->queued = 0;
        __syncthreads();
        uint32_t c[kSU], at[kSU];
        probe_hbm(region, next, 2u * L.r_len, lim, q, qr, wb, we, c, at, sh);
        if (queue) hand_off(heavy, hs, L.r_off, L.r_len);
        heavy_counts<kJoinBlock, kHeavyV, kOnePass>(rk + L.r_off, L.r_len, hs);
        uint64_t mine = 0;
#pragma unroll
        for (uint32_t u = 0; u < kSU; ++u) mine += is_heavy(c[u]) ? hs->cnt[c[u] & ~kHeavyBit] : c[u];
        const uint64_t pos0 = kOnePass ? block_reserve(mine, total, wtot, sb != 0) : base;
        base = write_round_hbm(next, rrp, qr, c, at, hs, pos0, capacity, out_r, out_s);
        heavy_writes<kJoinBlock, kHeavyV>(rk + L.r_off, rrp, L.r_len, hs, capacity, out_r, out_s);
        __syncthreads();  // the set is reused by the next round
    }
}

// The pairs of one work item (R_i in an LDS table, or its HBM table).
template <bool kOnePass, uint32_t RPT, bool kNt>
__device__ __forceinline__ void write_item(const ItemLoc L, uint32_t w, uint32_t* lds, uint64_t* wtot,
                                           const int32_t* __restrict__ rk, const int32_t* __restrict__ rr,
                                           const int32_t* __restrict__ sk, const int32_t* __restrict__ sr,
                                           uint32_t lds_cap, const uint64_t* __restrict__ ovf_table,
                                           const uint32_t* __restrict__ ovf_next, const HotKeys* hot,
                                           uint64_t base, unsigned long long* __restrict__ total,
                                           int32_t* __restrict__ out_r, int32_t* __restrict__ out_s,
                                           uint64_t capacity, HeavyQueue* heavy) {
    const int32_t* __restrict__ rrp = rr + L.r_off;
    const int32_t* __restrict__ skp = sk + L.s_begin;
    const int32_t* __restrict__ srp = sr + L.s_begin;
    int32_t q[kSU], qr[kSU];
    if (L.r_len <= lds_cap) {
        int32_t k[RPT];
        load_r<RPT>(rk + L.r_off, L.r_len, k);
        load_s<true, kNt>(skp, srp, w * kSubJ, min(w * kSubJ + kSubJ, L.s_n), q, qr);
        const LdsView v = lds_view(lds, lds_cap);
        const uint32_t log2H = table_log2H(L.r_len);
        build_lds<RPT>(k, L.r_len, log2H, v);
        for (uint32_t sb = 0; sb < L.s_n; sb += kJoinSub) {
            const uint32_t wb = sb + w * kSubJ, we = min(wb + kSubJ, L.s_n);
            if (sb) load_s<true, kNt>(skp, srp, wb, we, q, qr);
            uint32_t cf[kSU];
            int32_t rid0[kSU];
            probe_lds(v, log2H, q, wb, we, cf);
            fetch_first_rids(rrp, cf, rid0);
            const uint64_t pos0 = kOnePass ? block_reserve(lane_pairs_lds(cf), total, wtot, sb != 0) : base;
            base = write_round_lds(v, rrp, q, qr, cf, rid0, pos0, capacity, out_r, out_s);
        }
    } else {
        join_write_hbm<kOnePass>(L, w, rk, rrp, skp, srp, ovf_table, ovf_next, hot, base, total, wtot, out_r,
                                 out_s, capacity, reinterpret_cast<HbmLds*>(lds), heavy);
    }
}

// Polls of the item count by a helper workgroup before it leaves anyway (its
// help is only a speed-up: every queued chunk is also taken by the workgroup
// that queued it).
constexpr uint32_t kHelpWaitPolls = 1u << 20;
constexpr uint32_t kMaxHelpers = 256;

// A helper's loop: help with the queued tuples until the items the build
// counted are done.  Not inlined: inside the write kernel its registers cost
// the item path 6-10 us at 16M x 16M (measured), while as a call they do not.
__device__ __attribute__((noinline)) void help_until_done(HeavyQueue* heavy, const int32_t* rk, const int32_t* rr,
                                                         unsigned long long* total, uint64_t capacity, int32_t* out_r,
                                                         int32_t* out_s, uint32_t* lds, uint32_t* s_word) {
    const uint32_t expected = heavy->items_expected;
    for (uint32_t polls = 0;; ++polls) {
        __syncthreads();
        if (threadIdx.x == 0)
            *s_word = __hip_atomic_load(&heavy->items_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const bool all_done = *s_word >= expected;
        help_heavy<kJoinBlock>(heavy, rk, rr, total, capacity, out_r, out_s, lds);
        if (all_done || polls >= kHelpWaitPolls) break;
        __builtin_amdgcn_s_sleep(32);
    }
}

// Write pass.  kOnePass: instead of reading a scanned per-wave offset, each
// probe round reserves its pairs' output slots with block_reserve.  One-pass
// with `heavy`: every workgroup helps with the queued heavy tuples once its
// own item is written, and the grid has helper workgroups past item_grid.
// When the HBM-table build set heavy->wait (a partition may queue tuples), the
// items of such partitions count themselves done and the helpers keep helping
// until all of them are (the build counted them in items_expected), so that a
// tuple queued late still finds helpers; otherwise the helpers leave at once.
// (Counting every item instead cost the write ~0.26 ms at 16M x 16M: thousands
// of atomics on the queue's line, which every workgroup also reads.)  The helpers are at most half
// of the workgroups the device holds at once, so items always have room to
// run, whatever order the workgroups start in.
template <bool kOnePass, uint32_t RPT, bool kNt>
__global__ void __launch_bounds__(kJoinBlock) __attribute__((amdgpu_waves_per_eu(RPT > kRptMid ? 4 : 6)))
k_join_write(
    const PartPair* __restrict__ pairs, const uint32_t* __restrict__ item_begin,
    const ItemRec* __restrict__ item_rec, uint32_t P, const int32_t* __restrict__ rk,
    const int32_t* __restrict__ rr, const int32_t* __restrict__ sk, const int32_t* __restrict__ sr,
    uint32_t lds_cap, const uint64_t* __restrict__ ovf_table,
    const uint32_t* __restrict__ ovf_next, const HotKeys* __restrict__ hot, const uint64_t* __restrict__ wave_base,
    unsigned long long* __restrict__ total, int32_t* __restrict__ out_r, int32_t* __restrict__ out_s,
    uint64_t capacity, HeavyQueue* heavy, uint32_t item_grid) {
    extern __shared__ uint32_t lds[];
    __shared__ uint64_t wtot[kJoinWaves + 1];
    __shared__ uint32_t s_word;
    const uint32_t w = threadIdx.x / kWave;
    if (kOnePass && heavy && blockIdx.x >= item_grid) {  // a helper
        if (!heavy->wait) return;  // written by an earlier launch: uniform
        help_until_done(heavy, rk, rr, total, capacity, out_r, out_s, lds, &s_word);
        return;
    }
    const ItemLoc L = locate_item(item_rec);
    if (!L.live) return;
    const uint32_t item = L.item;
    const uint64_t base = kOnePass ? 0ull : wave_base[(uint64_t)item * kJoinWaves + w];
    write_item<kOnePass, RPT, kNt>(L, w, lds, wtot, rk, rr, sk, sr, lds_cap, ovf_table, ovf_next, hot, base, total,
                              out_r, out_s, capacity, heavy);
    // one-pass: help with the heavy tuples any workgroup queued (the LDS
    // tables are free now and give the scratch)
    if (kOnePass && heavy) {
        if (L.r_len > kHelpChunk) {  // an item the helpers wait for (the build counted it)
            __syncthreads();  // the item's hand-offs are made
            if (threadIdx.x == 0) atomicAdd(&heavy->items_done, 1u);
        }
        help_heavy<kJoinBlock>(heavy, rk, rr, total, capacity, out_r, out_s, lds);
    }
}

// Joins whose whole R fits one LDS table, several jobs per launch: one
// workgroup per (job, chunk of up to kJoinChunk S tuples) builds the table over
// the job's R and writes the chunk's pairs to the job's output with one-pass
// reservation.
template <uint32_t RPT>
__global__ void __launch_bounds__(kJoinBlock) __attribute__((amdgpu_waves_per_eu(RPT > kRptMid ? 4 : 6)))
k_direct_join(const DirectJob* __restrict__ jobs,
                                                           const uint32_t* __restrict__ item_job,
                                                           uint32_t lds_cap) {
    extern __shared__ uint32_t lds[];
    __shared__ uint64_t wtot[kJoinWaves + 1];
    const uint32_t w = threadIdx.x / kWave;
    const uint32_t item = xcd_remap(blockIdx.x, gridDim.x);
    const DirectJob J = jobs[item_job[item]];
    const uint32_t s_begin = (item - J.item0) * kJoinChunk;
    const uint32_t s_n = min(kJoinChunk, J.n_s - s_begin);
    const uint32_t r_len = min(J.n_r, lds_cap);  // the planner guarantees n_r <= lds_cap
    const int32_t* __restrict__ skp = J.sk + s_begin;
    const int32_t* __restrict__ srp = J.sr + s_begin;
    int32_t k[RPT];
    load_r<RPT>(J.rk, r_len, k);
    int32_t q[kSU], qr[kSU];
    load_s<true>(skp, srp, w * kSubJ, min(w * kSubJ + kSubJ, s_n), q, qr);
    const LdsView v = lds_view(lds, lds_cap);
    const uint32_t log2H = table_log2H(r_len);
    build_lds<RPT>(k, r_len, log2H, v);
    for (uint32_t sb = 0; sb < s_n; sb += kJoinSub) {
        const uint32_t wb = sb + w * kSubJ, we = min(wb + kSubJ, s_n);
        if (sb) load_s<true>(skp, srp, wb, we, q, qr);
        uint32_t cf[kSU];
        int32_t rid0[kSU];
        probe_lds(v, log2H, q, wb, we, cf);
        fetch_first_rids(J.rr, cf, rid0);
        const uint64_t pos0 = block_reserve(lane_pairs_lds(cf), (unsigned long long*)J.count, wtot, sb != 0);
        write_round_lds(v, J.rr, q, qr, cf, rid0, pos0, J.capacity, J.out_r, J.out_s);
    }
}

__global__ void k_direct_zero(const DirectJob* __restrict__ jobs, uint32_t njobs) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < njobs; j += gridDim.x * blockDim.x)
        *jobs[j].count = 0;
}

__global__ void k_direct_setup_one(DirectJob* job, uint32_t* item_job, DirectJob j, uint32_t nitems,
                                   uint64_t* err_clear) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *job = j;
        *j.count = 0;
        if (err_clear) *err_clear = 0;
    }
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nitems; i += gridDim.x * blockDim.x)
        item_job[i] = 0;
}

__global__ void k_write_zero(uint64_t* p, uint64_t* err_clear) {
    if (threadIdx.x == 0) {
        *p = 0;
        if (err_clear) *err_clear = 0;
    }
}

}  // namespace

size_t join_lds_bytes(uint32_t lds_cap, bool /*write*/) {
    static_assert(sizeof(HbmLds) <= sizeof(uint32_t) * (256 + 2 * kWave) + sizeof(uint64_t) * 256,
                  "the heavy-key set and the hot keys fit the smallest table area");
    return sizeof(uint32_t) * ((size_t)lds_cap + 2 * kWave) + sizeof(uint64_t) * lds_cap;
}

void direct_setup_one(DirectJob* job, uint32_t* item_job, const DirectJob& j, uint32_t nitems, Recorder& rec) {
    rec.before("direct_setup");
    hipLaunchKernelGGL(k_direct_setup_one, dim3(1), dim3(256), 0, rec.stream, job, item_job, j, nitems,
                       rec.err_clear);
    rec.after();
}

void direct_zero(const DirectJob* jobs, uint32_t njobs, Recorder& rec) {
    if (njobs == 0) return;
    rec.before("direct_zero");
    hipLaunchKernelGGL(k_direct_zero, dim3((njobs + 255) / 256), dim3(256), 0, rec.stream, jobs, njobs);
    rec.after();
}

static void allow_lds(const void* fn, size_t lds) {
    if (lds > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <uint32_t RPT>
void direct_join_t(const DirectJob* jobs, const uint32_t* item_job, uint32_t nitems, uint32_t lds_cap,
                   Recorder& rec) {
    const size_t lds = join_lds_bytes(lds_cap, true);
    allow_lds((const void*)k_direct_join<RPT>, lds);
    rec.before("direct_join");
    hipLaunchKernelGGL(k_direct_join<RPT>, dim3(nitems), dim3(kJoinBlock), lds, rec.stream, jobs, item_job,
                       lds_cap);
    rec.after();
}

void direct_join(const DirectJob* jobs, const uint32_t* item_job, uint32_t nitems, uint32_t lds_cap,
                 Recorder& rec) {
    if (nitems == 0) return;
    switch (join_rpt(lds_cap)) {
        case kRptSmall: direct_join_t<kRptSmall>(jobs, item_job, nitems, lds_cap, rec); break;
        case kRptMid: direct_join_t<kRptMid>(jobs, item_job, nitems, lds_cap, rec); break;
        default: direct_join_t<kRptLarge>(jobs, item_job, nitems, lds_cap, rec); break;
    }
}

void write_zero_count(uint64_t* d_count, Recorder& rec) {
    rec.before("zero_count");
    hipLaunchKernelGGL(k_write_zero, dim3(1), dim3(64), 0, rec.stream, d_count, rec.err_clear);
    rec.after();
}

// (an upper bound: the plan runs in workgroups of at least kMinPartBlock threads)
size_t plan_state_words(uint32_t P) { return 1 + plan_blocks(P, kMinPartBlock); }

uint32_t ovf_grid(uint32_t P, uint64_t n_r) {
    return (uint32_t)(P + (n_r + kOvfChunk - 1) / kOvfChunk);  // the smaller chunk bounds both
}

uint32_t join_grid(uint32_t P, uint64_t n_s) {
    const uint64_t items = P + (n_s + kJoinChunk - 1) / kJoinChunk;
    return (uint32_t)((items + 8 * kItemGroup - 1) / (8 * kItemGroup) * (8 * kItemGroup));  // item_of_block
}

void join_ovf_build(const PartPair* pairs, const uint32_t* ovf_begin, const uint32_t* ovf_part, uint32_t P,
                    uint32_t grid, const int32_t* rk, uint64_t* ovf_table, uint32_t* ovf_next, HotKeys* hot,
                    HeavyQueue* heavy, Recorder& rec, bool clear) {
    if (grid == 0) return;
    grid = grid < kOvfGrid ? grid : kOvfGrid;  // grid-stride: few chunks in the common case
    if (clear) {
        rec.before("ovf_clear");
        hipLaunchKernelGGL(k_ovf_clear, dim3(grid), dim3(256), 0, rec.stream, pairs, ovf_begin, ovf_part, P,
                           ovf_table);
        rec.after();
    }
    rec.before("ovf_build");
    hipLaunchKernelGGL(k_ovf_build, dim3(grid), dim3(256), 0, rec.stream, pairs, ovf_begin, ovf_part, P, rk,
                       ovf_table, ovf_next, hot, heavy);
    rec.after();
}

template <uint32_t RPT, bool kNt>
void join_count_t(const PartPair* pairs, const uint32_t* item_begin, const ItemRec* item_rec, uint32_t P,
                  uint32_t grid, const int32_t* rk, const int32_t* sk, uint32_t lds_cap, const uint64_t* ovf_table,
                  const uint32_t* ovf_next, const HotKeys* hot, uint64_t* wave_cnt, Recorder& rec) {
    const size_t lds = join_lds_bytes(lds_cap, false);
    allow_lds((const void*)k_join_count<RPT, kNt>, lds);
    rec.before("join_count");
    hipLaunchKernelGGL((k_join_count<RPT, kNt>), dim3(grid), dim3(kJoinBlock), lds, rec.stream, pairs, item_begin,
                       item_rec, P, rk, sk, lds_cap, ovf_table, ovf_next, hot, wave_cnt);
    rec.after();
}

template <bool kNt>
void join_count_n(const PartPair* pairs, const uint32_t* item_begin, const ItemRec* item_rec, uint32_t P,
                  uint32_t grid, const int32_t* rk, const int32_t* sk, uint32_t lds_cap, const uint64_t* ovf_table,
                  const uint32_t* ovf_next, const HotKeys* hot, uint64_t* wave_cnt, Recorder& rec) {
    switch (join_rpt(lds_cap)) {
        case kRptSmall:
            join_count_t<kRptSmall, kNt>(pairs, item_begin, item_rec, P, grid, rk, sk, lds_cap, ovf_table, ovf_next,
                                         hot, wave_cnt, rec);
            break;
        case kRptMid:
            join_count_t<kRptMid, kNt>(pairs, item_begin, item_rec, P, grid, rk, sk, lds_cap, ovf_table, ovf_next,
                                       hot, wave_cnt, rec);
            break;
        default:
            join_count_t<kRptLarge, kNt>(pairs, item_begin, item_rec, P, grid, rk, sk, lds_cap, ovf_table, ovf_next,
                                         hot, wave_cnt, rec);
            break;
    }
}

void join_count(const PartPair* pairs, const uint32_t* item_begin, const ItemRec* item_rec, uint32_t P,
                uint32_t grid,
                const int32_t* rk, const int32_t* sk, uint32_t lds_cap, const uint64_t* ovf_table,
                const uint32_t* ovf_next, const HotKeys* hot, uint64_t* wave_cnt, bool nt_s, Recorder& rec) {
    if (grid == 0) return;
    if (nt_s)
        join_count_n<true>(pairs, item_begin, item_rec, P, grid, rk, sk, lds_cap, ovf_table, ovf_next, hot,
                           wave_cnt, rec);
    else
        join_count_n<false>(pairs, item_begin, item_rec, P, grid, rk, sk, lds_cap, ovf_table, ovf_next, hot,
                            wave_cnt, rec);
}

template <bool kOnePass, uint32_t RPT, bool kNt>
void join_write_t(const PartPair* pairs, const uint32_t* item_begin, const ItemRec* item_rec, uint32_t P,
                  uint32_t grid, const int32_t* rk, const int32_t* rr, const int32_t* sk, const int32_t* sr,
                  uint32_t lds_cap, const uint64_t* ovf_table, const uint32_t* ovf_next, const HotKeys* hot,
                  const uint64_t* wave_base, uint64_t* total, int32_t* out_r, int32_t* out_s, uint64_t capacity,
                  HeavyQueue* heavy, Recorder& rec) {
    const size_t lds = join_lds_bytes(lds_cap, true);
    allow_lds((const void*)k_join_write<kOnePass, RPT, kNt>, lds);
    rec.before(kOnePass ? "join_write_1pass" : "join_write");
    const uint32_t item_grid = grid;
    if (kOnePass && heavy) {
        // helpers: at most half the workgroups resident at once (by LDS and by
        // the waves the register budget allows: 6 per SIMD, 4 for the large build)
        const uint32_t by_lds = (uint32_t)(160u * 1024u / (lds + 1024u));  // lds: this launch's dynamic bytes
        const uint32_t by_waves = (RPT > kRptMid ? 4u : 6u) * 4u / kJoinWaves;
        const uint32_t resident = 256u * std::max(1u, std::min(by_lds, by_waves));
        grid += std::max(1u, std::min(kMaxHelpers, resident / 2));
    }
    hipLaunchKernelGGL((k_join_write<kOnePass, RPT, kNt>), dim3(grid), dim3(kJoinBlock), lds, rec.stream, pairs,
                       item_begin, item_rec, P, rk, rr, sk, sr, lds_cap, ovf_table, ovf_next, hot, wave_base,
                       (unsigned long long*)total, out_r, out_s, capacity, heavy, item_grid);
    rec.after();
}

template <bool kOnePass, bool kNt>
void join_write_p(const PartPair* pairs, const uint32_t* item_begin, const ItemRec* item_rec, uint32_t P,
                  uint32_t grid, const int32_t* rk, const int32_t* rr, const int32_t* sk, const int32_t* sr,
                  uint32_t lds_cap, const uint64_t* ovf_table, const uint32_t* ovf_next, const HotKeys* hot,
                  const uint64_t* wave_base, uint64_t* total, int32_t* out_r, int32_t* out_s, uint64_t capacity,
                  HeavyQueue* heavy, Recorder& rec) {
    switch (join_rpt(lds_cap)) {
        case kRptSmall:
            join_write_t<kOnePass, kRptSmall, kNt>(pairs, item_begin, item_rec, P, grid, rk, rr, sk, sr, lds_cap,
                                              ovf_table, ovf_next, hot, wave_base, total, out_r, out_s, capacity, heavy, rec);
            break;
        case kRptMid:
            join_write_t<kOnePass, kRptMid, kNt>(pairs, item_begin, item_rec, P, grid, rk, rr, sk, sr, lds_cap,
                                            ovf_table, ovf_next, hot, wave_base, total, out_r, out_s, capacity, heavy, rec);
            break;
        default:
            join_write_t<kOnePass, kRptLarge, kNt>(pairs, item_begin, item_rec, P, grid, rk, rr, sk, sr, lds_cap,
                                              ovf_table, ovf_next, hot, wave_base, total, out_r, out_s, capacity, heavy, rec);
            break;
    }
}

void join_write(const PartPair* pairs, const uint32_t* item_begin, const ItemRec* item_rec, uint32_t P,
                uint32_t grid,
                const int32_t* rk, const int32_t* rr, const int32_t* sk, const int32_t* sr,
                uint32_t lds_cap, const uint64_t* ovf_table, const uint32_t* ovf_next,
                const uint64_t* wave_base, uint64_t* total, int32_t* out_r, int32_t* out_s,
                const HotKeys* hot, uint64_t capacity, HeavyQueue* heavy, bool nt_s, Recorder& rec) {
    if (grid == 0) return;
    if (wave_base == nullptr) {
        if (nt_s)
            join_write_p<true, true>(pairs, item_begin, item_rec, P, grid, rk, rr, sk, sr, lds_cap, ovf_table,
                                     ovf_next, hot, wave_base, total, out_r, out_s, capacity, heavy, rec);
        else
            join_write_p<true, false>(pairs, item_begin, item_rec, P, grid, rk, rr, sk, sr, lds_cap, ovf_table,
                                      ovf_next, hot, wave_base, total, out_r, out_s, capacity, heavy, rec);
    } else {
        if (nt_s)
            join_write_p<false, true>(pairs, item_begin, item_rec, P, grid, rk, rr, sk, sr, lds_cap, ovf_table,
                                      ovf_next, hot, wave_base, total, out_r, out_s, capacity, nullptr, rec);
        else
            join_write_p<false, false>(pairs, item_begin, item_rec, P, grid, rk, rr, sk, sr, lds_cap, ovf_table,
                                       ovf_next, hot, wave_base, total, out_r, out_s, capacity, nullptr, rec);
    }
}

}  // namespace hj
