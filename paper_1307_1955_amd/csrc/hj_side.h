// Work that rides along with another launch ("side jobs"): extra workgroups
// at the end of a radix-scatter grid run the next pass's setup or the join
// plan.  Both only read data that was complete before the hosting launch
// started (the histogram scan of the pass being scattered) and write tables
// that only later launches read, so they need no ordering with the scatter's
// own workgroups and cost no launch of their own.
#pragma once

#include "hj_device.h"
#include "hj_internal.h"

namespace hj {

constexpr uint32_t kMaxPlanWaves = 16;  // waves of the largest workgroup that runs the join plan

// Everything the pass-2 setup reads and writes.
struct Setup2Args {
    const uint32_t* hist1_scan;
    const uint32_t* tile_begin1;
    uint32_t bits1, n_r, n_s, tile, bits2, pad;
    const int32_t* key_in;
    const int32_t* rid_in;
    PartSeg* segs2;
    uint32_t* tile_begin2;
    uint32_t* tile_seg2;
};

// Everything the join plan reads and writes (see join_plan_block).
struct PlanArgs {
    const PartSeg* segs;
    const uint32_t* tile_begin;
    const uint32_t* hist_scan;
    uint32_t nseg, bits_last, n_r, n_s, total_bits, lds_cap;
    PartPair* pairs;
    uint32_t* item_begin;
    uint32_t* ovf_begin;
    ItemRec* item_rec;
    uint32_t* ovf_part;
    uint64_t* zero_total;
    uint64_t* state;
    // R's partition ranges from an earlier build (hj_build); nullptr: from the
    // histogram scan like S's
    const PartPair* r_pairs;
    ScanCtl ctl;  // the chained scan of the plan reports a give-up here
    // counted pass 2: final partition sizes (Reserve::tot) instead of hist_scan
    const uint32_t* tot;
    // records of item_rec up to here that have no item are written empty (the
    // join kernels' workgroup b takes record b)
    uint32_t items_ub;
};

enum SideKind : uint32_t { kSideNone = 0, kSideSetup2 = 1, kSidePlan = 2 };

struct SideJob {
    uint32_t kind;
    uint32_t blocks;  // extra workgroups at the end of the grid
    Setup2Args setup2;
    PlanArgs plan;
    // workgroups at the front of the grid (a multiple of 8) that sum count
    // rows (front == 0: none)
    uint32_t front, pad;
    CountSums sums;
};

// Join-plan workgroups of `block` threads (one partition pair per thread).
inline uint32_t plan_blocks(uint32_t P, uint32_t block) { return (P + block - 1) / block; }

// Start of final partition i of one relation (positions relative to the relation).
__device__ __forceinline__ uint32_t final_start(const PartSeg* __restrict__ segs,
                                                const uint32_t* __restrict__ tile_begin,
                                                const uint32_t* __restrict__ hist_scan, uint32_t rel,
                                                uint32_t nseg_rel, uint32_t bits_last, uint32_t i,
                                                uint32_t n_rel, uint32_t base_rel, uint32_t P) {
    if (i >= P) return n_rel;
    const uint32_t seg = rel * nseg_rel + (i >> bits_last);
    const uint32_t p = i & ((1u << bits_last) - 1u);
    const uint32_t nt = tile_begin[seg + 1] - tile_begin[seg];
    const uint32_t* hs = hist_scan + segs[seg].hist_base;
    const uint32_t r = nt ? hs[(uint64_t)p * nt] - hs[0] : 0u;
    return (uint32_t)(segs[seg].out_base - base_rel) + r;
}

__device__ __forceinline__ uint32_t items_of(const PartPair& pp) {
    return (pp.r_len && pp.s_len) ? (pp.s_len + kJoinChunk - 1) / kJoinChunk : 0u;
}

__device__ __forceinline__ uint32_t ovf_chunks_of(const PartPair& pp, uint32_t lds_cap) {
    const uint32_t chunk = ovf_chunk(pp.r_len);
    return (pp.r_len > lds_cap && pp.s_len) ? (pp.r_len + chunk - 1) / chunk : 0u;
}

// Final partition starts of a counted pass 2 for this workgroup's partitions
// i = blk * blockDim + threadIdx.x: R's in the low and S's in the high 32 bits
// (relative to each relation; R's left 0 with r_pairs).  Partition i is
// partition i mod 2^bits_last of segment i >> bits_last (one per pass-1
// partition), which starts at the segment's out_base; inside the segment the
// start is the sum of the totals of the partitions before it.  That sum is a
// block scan of the totals, less its value at the segment's first partition
// in the block, plus the totals of the segment's partitions in earlier blocks
// when the segment began before this block (2^bits_last > blockDim).
// `ex`: LDS of blockDim words of 64 bits.  Contains __syncthreads().
__device__ __forceinline__ uint64_t counted_starts(const PlanArgs& A, uint32_t blk, uint64_t* wt, uint64_t* ex,
                                                   uint64_t* v_out) {
    const uint32_t P = 1u << A.total_bits, b2 = A.bits_last;
    const uint32_t P1 = P >> b2;
    const uint32_t i0 = blk * blockDim.x, i = i0 + threadIdx.x;
    auto packed = [&](uint32_t j) -> uint64_t {
        return (A.r_pairs ? 0ull : (uint64_t)A.tot[j]) | (uint64_t)A.tot[P + j] << 32;
    };
    const uint64_t v = i < P ? packed(i) : 0ull;
    *v_out = v;
    // totals of the block's first segment that lie before the block
    const uint32_t seg_first = (i0 >> b2) << b2;
    uint64_t pre = 0;
    for (uint32_t j = seg_first + threadIdx.x; j < i0; j += blockDim.x) pre += packed(j);
    uint64_t pre_tot;
    (void)block_excl_scan(pre, wt, &pre_tot);
    uint64_t tot;
    const uint64_t e = block_excl_scan(v, wt, &tot);
    ex[threadIdx.x] = e;
    __syncthreads();
    const uint32_t s_i = max(i0, (i >> b2) << b2);  // first partition of i's segment in this block
    uint64_t within = e - ex[s_i - i0] + (s_i == i0 ? pre_tot : 0ull);
    __syncthreads();
    if (i >= P) return 0;
    const uint32_t q = i >> b2;
    const uint64_t r0 = A.r_pairs ? 0ull : A.segs[q].out_base + (uint32_t)within;
    const uint64_t s0 = A.segs[P1 + q].out_base - A.n_r + (uint32_t)(within >> 32);
    return (uint64_t)(uint32_t)r0 | (uint64_t)(uint32_t)s0 << 32;
}

// Plan (one thread per partition pair, workgroups in ticket order): ranges of
// R_i and S_i from the last pass's histogram scan (or a counted pass 2's
// totals), the pair's work items and HBM-table build chunks, their exclusive
// scans over all pairs (one chained scan of both counts packed in one word),
// the work-item records and the chunk -> pair map.
// state[0]: ticket; state[1 + b]: status of workgroup b (cleared beforehand).
// Run by plan_blocks(P, blockDim.x) workgroups.  `lds`: blockDim words of 64
// bits of scratch (a counted pass 2).
__device__ __forceinline__ void join_plan_block(const PlanArgs& A, uint64_t* lds) {
    const PartSeg* __restrict__ segs = A.segs;
    const uint32_t* __restrict__ tile_begin = A.tile_begin;
    const uint32_t nseg = A.nseg, bits_last = A.bits_last, n_r = A.n_r, n_s = A.n_s;
    const uint32_t total_bits = A.total_bits, lds_cap = A.lds_cap;
    const uint32_t* __restrict__ hist_scan = A.hist_scan;
    PartPair* __restrict__ pairs = A.pairs;
    uint32_t* __restrict__ item_begin = A.item_begin;
    uint32_t* __restrict__ ovf_begin = A.ovf_begin;
    ItemRec* __restrict__ item_rec = A.item_rec;
    uint32_t* __restrict__ ovf_part = A.ovf_part;
    uint64_t* __restrict__ zero_total = A.zero_total;
    uint64_t* state = A.state;
    __shared__ uint64_t wt[kMaxPlanWaves];
    __shared__ uint32_t s_blk;
    __shared__ uint64_t s_prefix;
    if (threadIdx.x == 0) s_blk = (uint32_t)atomicAdd((unsigned long long*)state, 1ull);
    __syncthreads();
    const uint32_t blk = s_blk;
    const uint32_t P = 1u << total_bits;
    const uint32_t nseg_rel = nseg / 2;
    const uint32_t i = blk * blockDim.x + threadIdx.x;
    if (i == 0 && zero_total) *zero_total = 0;
    PartPair pp{0, 0, 0, 0};
    uint32_t ni = 0, no = 0;
    if (A.tot) {  // uniform
        uint64_t v;
        const uint64_t st = counted_starts(A, blk, wt, lds, &v);
        if (i < P) {
            // clamped: a partition never extends past its relation
            const uint32_t s0 = min((uint32_t)(st >> 32), n_s);
            pp.s_off = s0;
            pp.s_len = min(s0 + (uint32_t)(v >> 32), n_s) - s0;
            if (A.r_pairs) {
                const PartPair q = A.r_pairs[i];
                pp.r_off = q.r_off;
                pp.r_len = q.r_len;
            } else {
                const uint32_t r0 = min((uint32_t)st, n_r);
                pp.r_off = r0;
                pp.r_len = min(r0 + (uint32_t)v, n_r) - r0;
            }
            ni = items_of(pp);
            no = ovf_chunks_of(pp, lds_cap);
        }
    } else if (i < P) {
        const uint32_t s0 = min(final_start(segs, tile_begin, hist_scan, 1, nseg_rel, bits_last, i, n_s, n_r, P), n_s);
        // clamped: a partition never extends past its relation or runs backwards
        const uint32_t s1 = max(s0, min(final_start(segs, tile_begin, hist_scan, 1, nseg_rel, bits_last, i + 1, n_s, n_r, P), n_s));
        if (A.r_pairs) {
            const PartPair q = A.r_pairs[i];
            pp.r_off = q.r_off;
            pp.r_len = q.r_len;
        } else {
            const uint32_t r0 = min(final_start(segs, tile_begin, hist_scan, 0, nseg_rel, bits_last, i, n_r, 0, P), n_r);
            const uint32_t r1 = max(r0, min(final_start(segs, tile_begin, hist_scan, 0, nseg_rel, bits_last, i + 1, n_r, 0, P), n_r));
            pp.r_off = r0;
            pp.r_len = r1 - r0;
        }
        pp.s_off = s0;
        pp.s_len = s1 - s0;
        ni = items_of(pp);
        no = ovf_chunks_of(pp, lds_cap);
    }
    // items and chunks are each below 2^31: packed as items | chunks << 31
    uint64_t tot;
    const uint64_t excl = block_excl_scan((uint64_t)ni | ((uint64_t)no << 31), wt, &tot);
    if (threadIdx.x < kWave) {
        const uint64_t prefix = lookback_wave(state + 1, blk, tot, A.ctl);
        if (threadIdx.x == 0) s_prefix = prefix;
    }
    __syncthreads();
    const uint64_t run = s_prefix + excl;
    const uint32_t ib = (uint32_t)(run & 0x7FFFFFFFu), ob = (uint32_t)(run >> 31);
    if (i < P) {
        pairs[i] = pp;
        item_begin[i] = ib;
        ovf_begin[i] = ob;
        for (uint32_t x = 0; x < ni; ++x)
            item_rec[ib + x] = ItemRec{pp.r_off, pp.r_len, pp.s_off + x * kJoinChunk,
                                       min(kJoinChunk, pp.s_len - x * kJoinChunk)};
        for (uint32_t x = 0; x < no; ++x) ovf_part[ob + x] = i;
    }
    if (i == P - 1) {  // the last pair also writes the totals
        item_begin[P] = ib + ni;
        ovf_begin[P] = ob + no;
    }
    // the workgroup of the last pair marks the records past the last item empty
    __shared__ uint32_t s_live;
    const bool last_blk = blk * blockDim.x <= P - 1 && P - 1 < (blk + 1) * blockDim.x;  // uniform
    if (last_blk) {
        if (i == P - 1) s_live = ib + ni;
        __syncthreads();
        for (uint32_t x = s_live + threadIdx.x; x < A.items_ub; x += blockDim.x) item_rec[x] = ItemRec{0, 0, 0, 0};
    }
}



// Start of partition q of a pass-1 segment relative to the segment.
__device__ __forceinline__ uint32_t seg_part_start(const uint32_t* __restrict__ hs_seg, uint32_t nt,
                                                   uint32_t q) {
    return nt ? hs_seg[(uint64_t)q * nt] - hs_seg[0] : 0u;
}

// Pass-2 segment table (every pass-1 partition of R and of S), its tile
// offsets and the tile -> segment map, from the pass-1 histogram scan.  Run by
// one workgroup of any size; `lds` holds lds_words scratch words (the segment
// tile offsets are kept there for the tile map when they fit).
__device__ __forceinline__ void setup_pass2_block(const Setup2Args& A, uint32_t* lds, uint32_t lds_words) {
    const uint32_t* __restrict__ hist1_scan = A.hist1_scan;
    const uint32_t* __restrict__ tile_begin1 = A.tile_begin1;
    const uint32_t bits1 = A.bits1, n_r = A.n_r, n_s = A.n_s, tile = A.tile, bits2 = A.bits2;
    const int32_t* key_in = A.key_in;
    const int32_t* rid_in = A.rid_in;
    PartSeg* __restrict__ segs2 = A.segs2;
    uint32_t* __restrict__ tile_begin2 = A.tile_begin2;
    uint32_t* __restrict__ tile_seg2 = A.tile_seg2;
    uint32_t* wt = lds;                   // [kScanScratch]
    uint32_t* tb = lds + kScanScratch;    // [nseg + 1] when it fits
    const uint32_t P1 = 1u << bits1;
    const uint32_t nseg = 2 * P1;
    const uint32_t per = (nseg + blockDim.x - 1) / blockDim.x;
    const uint32_t a = threadIdx.x * per;
    const uint32_t b = min(a + per, nseg);
    const uint32_t nt_r = tile_begin1[1], nt_s = tile_begin1[2] - tile_begin1[1];
    // pass 1 used hist_base = 0 for R and nt_r << bits1 for S
    auto seg_range = [&](uint32_t s, uint32_t* off, uint32_t* len, uint32_t* base) {
        const uint32_t rel = s >= P1;
        const uint32_t q = s - rel * P1;
        const uint32_t nt = rel ? nt_s : nt_r;
        const uint32_t* hs = hist1_scan + (rel ? ((uint64_t)nt_r << bits1) : 0ull);
        const uint32_t n = rel ? n_s : n_r;
        // clamped so a segment always lies inside its relation
        const uint32_t st = min(seg_part_start(hs, nt, q), n);
        const uint32_t en = max(st, q + 1 < P1 ? min(seg_part_start(hs, nt, q + 1), n) : n);
        *off = st;
        *len = en - st;
        *base = rel ? n_r : 0u;
    };
    uint32_t ntiles = 0;
    for (uint32_t s = a; s < b; ++s) {
        uint32_t off, len, base;
        seg_range(s, &off, &len, &base);
        ntiles += (len + tile - 1) / tile;
    }
    uint32_t total;
    uint32_t run = block_excl_scan(ntiles, wt, &total);
    const bool in_lds = nseg + 1 + kScanScratch <= lds_words;
    for (uint32_t s = a; s < b; ++s) {
        uint32_t off, len, base;
        seg_range(s, &off, &len, &base);
        PartSeg g;
        g.key_in = key_in + base + off;
        g.rid_in = rid_in + base + off;
        g.out_base = (uint64_t)base + off;
        g.hist_base = (uint64_t)run << bits2;
        g.n = len;
        g.pad = 0;
        segs2[s] = g;
        tile_begin2[s] = run;
        if (in_lds) tb[s] = run;
        const uint32_t nt = (len + tile - 1) / tile;
        if (!in_lds)
            for (uint32_t x = 0; x < nt; ++x) tile_seg2[run + x] = s;
        run += nt;
    }
    if (threadIdx.x == 0) {
        tile_begin2[nseg] = total;
        if (in_lds) tb[nseg] = total;
    }
    if (in_lds) {
        // every thread maps its share of the tiles to segments (binary search in LDS)
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < total; t += blockDim.x) tile_seg2[t] = upper_index(tb, nseg, t);
    }
}


// Workgroup b of the count-row sums (CountSums): rows [row0, row1) of one
// relation and cw 16-count columns, each column summed in registers by
// `phases` threads (16-byte loads, eight rows in flight per thread), the
// phases combined in LDS (when `lds` holds cw * 16 words), then added to the
// totals; and the escapes of those rows that fall in the columns.
__device__ __forceinline__ void sum_count_rows(const CountSums& A, uint32_t b, uint32_t* lds,
                                               uint32_t lds_words) {
    const uint32_t PA = 1u << A.bits;
    const uint32_t C = PA / 16;
    const uint32_t cw = min(C, (uint32_t)blockDim.x), phases = blockDim.x / cw;
    const uint32_t cg = count_sum_groups(A.bits, blockDim.x);
    const uint32_t rg_r = (A.nt_r + A.rows_per - 1) / A.rows_per;
    const uint32_t rg_s = (A.nt_s + A.rows_per - 1) / A.rows_per;
    const uint32_t q = b / cg;
    if (q >= rg_r + rg_s) return;  // rounding workgroups (uniform)
    const uint32_t rel = q >= rg_r;
    const uint32_t first = rel ? A.nt_r : 0u, last = rel ? A.nt_r + A.nt_s : A.nt_r;
    const uint32_t row0 = first + (q - (rel ? rg_r : 0u)) * A.rows_per;
    const uint32_t row1 = min(row0 + A.rows_per, last);
    if (row0 >= row1) return;  // uniform
    const uint32_t lo = (b % cg) * cw * 16;  // first count of the column group
    const uint32_t col = threadIdx.x % cw, ph = threadIdx.x / cw;
    const uint32_t n = row1 - row0;
    uint32_t acc[16];
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) acc[e] = 0;
    if (ph < phases) {
        const uint4* __restrict__ src = reinterpret_cast<const uint4*>(A.rows) + (uint64_t)row0 * C + lo / 16 + col;
#pragma unroll 8
        for (uint32_t r = ph; r < n; r += phases) {
            const uint4 w = src[(uint64_t)r * C];
            const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (uint32_t k = 0; k < 16; ++k) acc[k] += (ws[k / 4] >> (8 * (k % 4))) & 0xFFu;
        }
    }
    uint32_t* __restrict__ tot = A.tot + (uint64_t)rel * PA;
    if (phases > 1 && cw * 16 <= lds_words) {  // uniform
        for (uint32_t i = threadIdx.x; i < cw * 16; i += blockDim.x) lds[i] = 0;
        __syncthreads();
#pragma unroll
        for (uint32_t e = 0; e < 16; ++e)
            if (acc[e]) atomicAdd(&lds[col * 16 + e], acc[e]);
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cw * 16; i += blockDim.x) {
            const uint32_t v = lds[i];
            if (v) atomicAdd(&tot[lo + i], v);
        }
    } else {
#pragma unroll
        for (uint32_t e = 0; e < 16; ++e)
            if (acc[e]) atomicAdd(&tot[lo + col * 16 + e], acc[e]);
    }
    for (uint32_t i = threadIdx.x; i < n * kCountEsc; i += blockDim.x) {
        const uint32_t v = A.esc[(uint64_t)row0 * kCountEsc + i];
        const uint32_t c = v & 0x3FFFu, bin = v >> 14;
        if (c && bin >= lo && bin < lo + cw * 16) atomicAdd(&tot[bin], c);
    }
}

// Runs the side job on workgroup `b` of its extra workgroups.  `lds`: the
// hosting kernel's dynamic LDS (lds_words words).
__device__ __forceinline__ void run_side_job(const SideJob& J, uint32_t b, uint32_t* lds, uint32_t lds_words) {
    if (J.kind == kSideSetup2) {
        if (b == 0) setup_pass2_block(J.setup2, lds, lds_words);
    } else if (J.kind == kSidePlan) {
        join_plan_block(J.plan, reinterpret_cast<uint64_t*>(lds));
    }
}

}  // namespace hj
