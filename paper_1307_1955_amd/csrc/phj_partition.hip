// Radix partitioning for the partitioned hash join (Algorithm 2, "Partition",
// steps n1-n3; Section 3.1: passes on the low bits of the integer hash value).
//
// A pass works on a list of segments (pass 1: R and S; pass 2: every pass-1
// partition of R and of S) cut into tiles of `tile` tuples.  Per tile:
//   hist     n1: partition number of every tuple, counted with LDS atomics
//            (at low fan-out the tuples of one wave that share a partition are
//            grouped with one ballot per radix bit and their leader adds the
//            group size); the tile's counters go to
//            hist[segment block + p * ntiles + tile].
//   scan     (scan.hip) exclusive scan of hist: partition-major inside each
//            segment, so each (partition, tile) run has one global offset.
//   scatter  n2-n3: the tile is re-read, every tuple gets its rank inside its
//            partition (value returned by its LDS atomic, or leader atomic +
//            popcount of lower group lanes at low fan-out), the tile is
//            reordered by partition in LDS and written out run by run, so
//            consecutive lanes store to consecutive addresses.
// Counted pass 2 (two passes of 4..13 bits in all): the pass-1 hist also counts
// every tuple's final partition and writes them as a row of 8-bit counts per
// tile (larger counts as escapes); workgroups at the front of the pass-1
// scatter sum the rows into per-segment totals, and each pass-2 scatter tile
// reserves its run of every partition on a per-partition cursor instead of
// reading a pass-2 histogram scan.  Tiles of large joins are read with
// non-temporal loads (PassCfg::nt).
// The paper's partition "buckets" with dynamically allocated storage
// (Section 3.1, Section 3.3) become contiguous partitions at counted offsets.
#include "hj_device.h"
#include "hj_internal.h"
#include "hj_side.h"

namespace hj {

namespace {

// Up to this many radix bits (8 partitions) the lanes of a wave that share a
// partition are grouped with ballots and one leader atomic per group: at such
// low fan-out most lanes of a wave hit the same few LDS counters.  Above it,
// one LDS atomic per tuple is faster on gfx950 (measured at 64 partitions:
// histogram 2x, scatter 1.2x).
constexpr uint32_t kBallotMaxBits = 3;

struct TileLoc {
    uint32_t seg, tl, nt, start, len;
};

// tile_seg (optional): the segment of every tile, written by the pass's setup
// kernel; without it the segment is found by binary search over tile_begin.
__device__ __forceinline__ TileLoc locate(const PartSeg* __restrict__ segs,
                                          const uint32_t* __restrict__ tile_begin,
                                          const uint32_t* __restrict__ tile_seg, uint32_t nseg,
                                          uint32_t tile, uint32_t T) {
    TileLoc t;
    t.seg = tile_seg ? tile_seg[tile] : upper_index(tile_begin, nseg, tile);
    const uint32_t b0 = tile_begin[t.seg];
    t.tl = tile - b0;
    t.nt = tile_begin[t.seg + 1] - b0;
    t.start = t.tl * T;
    const uint32_t n = segs[t.seg].n;
    t.len = min(T, n - t.start);
    return t;
}

__device__ __forceinline__ uint32_t part_of(int32_t key, const PassCfg& c) {
    return (radix_hash(key, c.hash_kind) >> c.shift) & ((1u << c.bits) - 1u);
}

// Lanes of this wave whose `p` equals this lane's (only lanes with `valid`).
__device__ __forceinline__ uint64_t match_mask(uint32_t p, uint32_t bits, bool valid) {
    uint64_t m = __ballot(valid);
    for (uint32_t b = 0; b < bits; ++b) {
        const bool bit = (p >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        m &= bit ? bal : ~bal;
    }
    return valid ? m : 0ull;
}

// Loads the elements [0, len) of a tile (len <= BLOCK * IPT) that starts
// at `p` (4-byte aligned) with 16-byte vector loads: lane-contiguous 16-byte
// chunks of the enclosing aligned window; thread t, slot k holds chunk
// t + k * BLOCK, i.e. v[4k + e] = window element 4 (t + k BLOCK) + e,
// tile element that minus the misalignment s = (p mod 16) / 4.  Only chunks lying
// wholly inside the tile are read as vectors; the elements of the (at most two)
// partial chunks are read one by one, and the up to 3 tile elements past the
// window (when s > 0) go to `x` of threads 0..2.  Nothing outside the tile is
// read.  Returns the validity mask: bit i for v[i], bit 4 IPT for x.  Element
// order inside a tile is free: counts and ranks do not depend on it.
// Pointers into device memory taken from tables in memory are generic; read
// through the global address space the loads are global loads, which unlike
// generic (flat) ones are not counted against LDS accesses (a wait for LDS
// would otherwise also wait for the tile's loads).  kStream: the vector loads
// are marked non-temporal (PassCfg::nt, large joins: each launch reads its
// input once).
typedef __attribute__((address_space(1))) const int32_t gint32;
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const i32x4 gi32x4;

template <uint32_t BLOCK, uint32_t IPT, bool kStream = false>
__device__ __forceinline__ uint64_t load_tile_vec(const int32_t* __restrict__ pg, uint32_t len, int32_t* v,
                                                  int32_t& x) {
    static_assert(IPT % 4 == 0 && IPT <= 32, "vector tile slots");
    gint32* __restrict__ p = (gint32*)pg;
    const uint32_t s = (uint32_t)(((uintptr_t)pg >> 2) & 3u);
    gint32* __restrict__ q = p - s;  // 16-byte aligned
    uint64_t valid = 0;
#pragma unroll
    for (uint32_t k = 0; k < IPT / 4; ++k) {
        const uint32_t c = threadIdx.x + k * BLOCK;
        const int32_t i0 = (int32_t)(4 * c) - (int32_t)s;  // tile index of the chunk's first element
        if (i0 >= 0 && i0 + 4 <= (int32_t)len) {
            gi32x4* a = reinterpret_cast<gi32x4*>(q + 4 * c);
            const i32x4 w = kStream ? __builtin_nontemporal_load(a) : *a;
            v[4 * k] = w.x;
            v[4 * k + 1] = w.y;
            v[4 * k + 2] = w.z;
            v[4 * k + 3] = w.w;
            valid |= 0xFull << (4 * k);
        } else {
#pragma unroll
            for (uint32_t e = 0; e < 4; ++e) {
                const int32_t i = i0 + (int32_t)e;
                const bool ok = i >= 0 && i < (int32_t)len;
                v[4 * k + e] = ok ? q[4 * c + e] : 0;
                valid |= (uint64_t)ok << (4 * k + e);
            }
        }
    }
    const uint32_t xi = BLOCK * IPT - s + threadIdx.x;  // past the window
    const bool xok = threadIdx.x < s && xi < len;
    x = xok ? p[xi] : 0;
    valid |= (uint64_t)xok << IPT;
    return valid;
}

// The pass-1 set-up that later launches read (see Pass1), by one workgroup.
__device__ __forceinline__ void pass1_setup(const Pass1& A) {
    for (uint64_t i = threadIdx.x; i < A.nzero; i += blockDim.x) A.zero[i] = 0;
    if (threadIdx.x == 0) {
        if (A.err_clear) *A.err_clear = 0;
        PartSeg a;
        a.key_in = A.rk; a.rid_in = A.rr; a.out_base = 0; a.hist_base = 0; a.n = A.n_r; a.pad = 0;
        PartSeg b;
        b.key_in = A.sk; b.rid_in = A.sr; b.out_base = A.n_r; b.hist_base = A.hist_s; b.n = A.n_s; b.pad = 0;
        A.segs[0] = a;
        A.segs[1] = b;
        A.tile_begin[0] = 0;
        A.tile_begin[1] = A.nt_r;
        A.tile_begin[2] = A.ntiles;
    }
}

// kPass1: the tiles of R and S from the launch arguments (p1), and workgroup 0
// also does the pass's set-up; else the segments in memory.  kCount (pass 1 of
// a counted pass 2): the tile's counts per final partition are also written,
// as row p1.rows + tile * 2^bits_all of 8-bit counts and the tile's escapes.
template <uint32_t BLOCK, uint32_t IPT, bool kPass1, bool kCount, bool kNt>
__global__ void __launch_bounds__(BLOCK) k_part_hist(const PartSeg* __restrict__ segs,
                                                         const uint32_t* __restrict__ tile_begin,
                                                         const uint32_t* __restrict__ tile_seg,
                                                         uint32_t nseg, PassCfg cfg,
                                                         uint32_t* __restrict__ hist, Pass1 p1) {
    static_assert(kPass1 || !kCount, "counting rides on pass 1");
    extern __shared__ uint32_t lds[];
    constexpr uint32_t T = BLOCK * IPT;
    uint32_t* cnt = lds;
    const uint32_t P = 1u << cfg.bits;
    const uint32_t PA = kCount ? 1u << p1.bits_all : 0u;
    // [PA] (kCount): count of final partition i at (i mod 16) * PA / 16 + i / 16,
    // so that the 16 counts one thread packs into a store lie in 16 banks
    // apart from its neighbours'
    uint32_t* cnt_all = lds + P;
    const uint32_t sh_all = kCount ? p1.bits_all - 4 : 0u;
    uint32_t* esc = cnt_all + PA;  // [kCountEsc] escapes, then their number (kCount)
    static_assert(!kCount || T < (kCountEsc + 1) * kCountEscMin, "escapes of a tile fit its list");
    const int32_t* __restrict__ kin;
    uint32_t len, tl, nt;
    uint64_t hist_base;
    uint32_t row = 0;
    if (kPass1) {
        if (blockIdx.x == 0) pass1_setup(p1);
        const uint32_t tile = live_remap(blockIdx.x, p1.ntiles);
        if (tile >= p1.ntiles) return;
        row = tile;
        const bool s1 = tile >= p1.nt_r;  // field by field: no dynamic index into the arguments
        tl = s1 ? tile - p1.nt_r : tile;
        nt = s1 ? p1.ntiles - p1.nt_r : p1.nt_r;
        len = min(T, (s1 ? p1.n_s : p1.n_r) - tl * T);
        kin = (s1 ? p1.sk : p1.rk) + tl * T;
        hist_base = s1 ? p1.hist_s : 0ull;
    } else {
        const uint32_t ntiles = tile_begin[nseg];
        const uint32_t tile = live_remap(blockIdx.x, ntiles);
        if (tile >= ntiles) return;
        const TileLoc t = locate(segs, tile_begin, tile_seg, nseg, tile, T);
        const PartSeg sg = segs[t.seg];
        kin = sg.key_in + t.start;
        len = t.len;
        tl = t.tl;
        nt = t.nt;
        hist_base = sg.hist_base;
    }
    int32_t keys[IPT], kx;
    const uint64_t valid = load_tile_vec<BLOCK, IPT, kNt>(kin, len, keys, kx);
    // kCount with pass 1 above at least 4 low bits (b2 >= 4): the 16 final
    // partitions of a packed column below share their pass-1 partition (the
    // column index >> (b2 - 4)), so the pass-1 counts are summed from the
    // columns, one LDS atomic per column instead of one per tuple (uniform)
    const bool from_cols = kCount && cfg.shift >= 4;
    // counters cleared while the tile's loads are in flight
    for (uint32_t i = threadIdx.x; i < P; i += BLOCK) cnt[i] = 0;
    if (kCount)
        for (uint32_t i = threadIdx.x; i < PA + kCountEsc + 1; i += BLOCK) cnt_all[i] = 0;
    __syncthreads();
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (uint32_t k = 0; k < IPT; ++k) {
        const bool ok = (valid >> k) & 1u;
        const uint32_t h = radix_hash(keys[k], cfg.hash_kind);
        const uint32_t p = (h >> cfg.shift) & (P - 1u);
        if (kCount && ok) atomicAdd(&cnt_all[((h & 15u) << sh_all) | ((h & (PA - 1u)) >> 4)], 1u);
        if (!from_cols) {
            if (cfg.bits <= kBallotMaxBits) {
                const uint64_t m = match_mask(p, cfg.bits, ok);
                if (ok && (m & lt) == 0) atomicAdd(&cnt[p], (uint32_t)__popcll(m));
            } else if (ok) {
                atomicAdd(&cnt[p], 1u);
            }
        }
    }
    if ((valid >> IPT) & 1u) {
        const uint32_t h = radix_hash(kx, cfg.hash_kind);
        if (!from_cols) atomicAdd(&cnt[(h >> cfg.shift) & (P - 1u)], 1u);
        if (kCount) atomicAdd(&cnt_all[((h & 15u) << sh_all) | ((h & (PA - 1u)) >> 4)], 1u);
    }
    __syncthreads();
    uint32_t* __restrict__ h = hist + hist_base + tl;
    if (!from_cols)
        for (uint32_t p = threadIdx.x; p < P; p += BLOCK) h[(uint64_t)p * nt] = cnt[p];
    if (kCount) {
        // 16 counts per 16-byte store (PA >= 16); counts from kCountEscMin on
        // are 0 here and escaped
        uint4* __restrict__ out = reinterpret_cast<uint4*>(p1.rows + (uint64_t)row * PA);
        for (uint32_t c = threadIdx.x; c < PA / 16; c += BLOCK) {
            uint32_t w[4], sum = 0;
#pragma unroll
            for (uint32_t q = 0; q < 4; ++q) {
                w[q] = 0;
#pragma unroll
                for (uint32_t e = 0; e < 4; ++e) {
                    uint32_t x = cnt_all[((4 * q + e) << sh_all) + c];  // partition 16 c + 4 q + e
                    sum += x;
                    if (x >= kCountEscMin) {
                        const uint32_t k = atomicAdd(&esc[kCountEsc], 1u);
                        if (k < kCountEsc) esc[k] = (16 * c + 4 * q + e) << 14 | x;
                        x = 0;
                    }
                    w[q] |= x << (8 * e);
                }
            }
            out[c] = make_uint4(w[0], w[1], w[2], w[3]);
            if (from_cols && sum) atomicAdd(&cnt[c >> (cfg.shift - 4)], sum);
        }
        __syncthreads();
        if (from_cols)
            for (uint32_t p = threadIdx.x; p < P; p += BLOCK) h[(uint64_t)p * nt] = cnt[p];
        if (threadIdx.x < kCountEsc) p1.esc[(uint64_t)row * kCountEsc + threadIdx.x] = esc[threadIdx.x];
    }
}

template <uint32_t BLOCK, uint32_t IPT, bool kNt>
__global__ void __launch_bounds__(BLOCK) k_part_scatter(const PartSeg* __restrict__ segs,
                                                            const uint32_t* __restrict__ tile_begin,
                                                            const uint32_t* __restrict__ tile_seg,
                                                            uint32_t nseg, PassCfg cfg,
                                                            const uint32_t* __restrict__ hist_scan,
                                                            int32_t* __restrict__ key_out,
                                                            int32_t* __restrict__ rid_out, SideJob side,
                                                            uint32_t lds_words, Reserve rsv) {
    extern __shared__ uint32_t lds[];
    if (blockIdx.x >= gridDim.x - side.blocks) {  // extra workgroups: the side job
        run_side_job(side, blockIdx.x - (gridDim.x - side.blocks), lds, lds_words);
        return;
    }
    if (blockIdx.x < side.front) {  // count-row sums at the front
        sum_count_rows(side.sums, blockIdx.x, lds, lds_words);
        return;
    }
    const uint32_t blk = blockIdx.x - side.front;  // (front is a multiple of 8: same XCD)
    constexpr uint32_t T = BLOCK * IPT;
    const uint32_t P = 1u << cfg.bits;
    const uint32_t Pp = P < kWave ? kWave : P;  // scan length, a multiple of 64
    const bool counted = rsv.tot != nullptr;    // uniform
    uint32_t* cnt = lds;                         // [Pp]  counts, then local starts
    uint32_t* delta = cnt + Pp;                  // [P]   global offset - local start
    uint32_t* ctot = delta + Pp;                 // [kScanScratch]
    int32_t* skey = (int32_t*)(ctot + kScanScratch);  // [T]
    int32_t* srid = skey + T;                        // [T]
    uint32_t* resv = (uint32_t*)(srid + T);          // [Pp] (counted, P > BLOCK): reserved offsets

    const uint32_t ntiles = tile_begin[nseg];
    const uint32_t tile = live_remap(blk, ntiles);
    if (tile >= ntiles) return;
    const TileLoc t = locate(segs, tile_begin, tile_seg, nseg, tile, T);
    const PartSeg sg = segs[t.seg];
    const int32_t* __restrict__ kin = sg.key_in + t.start;
    const int32_t* __restrict__ rin = sg.rid_in + t.start;
    int32_t keys[IPT], rids[IPT], kx, rx;
    uint32_t rank[IPT];
    uint64_t valid;
    if ((((uintptr_t)kin ^ (uintptr_t)rin) & 15u) == 0) {  // same misalignment: one vector pattern for both
        valid = load_tile_vec<BLOCK, IPT, kNt>(kin, t.len, keys, kx);
        load_tile_vec<BLOCK, IPT, kNt>(rin, t.len, rids, rx);
    } else {
        valid = 0;
#pragma unroll
        for (uint32_t k = 0; k < IPT; ++k) {
            const uint32_t idx = k * BLOCK + threadIdx.x;
            const bool ok = idx < t.len;
            keys[k] = ok ? ((gint32*)kin)[idx] : 0;
            rids[k] = ok ? ((gint32*)rin)[idx] : 0;
            valid |= (uint64_t)ok << k;
        }
        kx = rx = 0;
        // awaited here: the compiler joins this branch into the vector one
        // behind a flag, and loads still in flight on it would put waits
        // between the vector loads of the other
#pragma unroll
        for (uint32_t k = 0; k < IPT; ++k) {
            settle((uint32_t)keys[k]);
            settle((uint32_t)rids[k]);
        }
    }
    // This tile's global partition offsets (counted: its segment's totals) do
    // not depend on the tile's data: fetched together with it (first BLOCK
    // partitions; the rest later).
    const uint32_t* __restrict__ hs = counted ? rsv.tot + (uint64_t)t.seg * P : hist_scan + sg.hist_base;
    const uint32_t hs_own = threadIdx.x < P ? hs[counted ? threadIdx.x : (uint64_t)threadIdx.x * t.nt + t.tl] : 0u;
    const uint32_t seg0 = counted ? 0u : hs[0];
    // counters cleared while the loads are in flight
    for (uint32_t i = threadIdx.x; i < Pp; i += BLOCK) cnt[i] = 0;
    __syncthreads();
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (uint32_t k = 0; k < IPT; ++k) {
        const bool ok = (valid >> k) & 1u;
        const uint32_t p = part_of(keys[k], cfg);
        if (cfg.bits <= kBallotMaxBits) {
            const uint64_t m = match_mask(p, cfg.bits, ok);
            const uint32_t below = (uint32_t)__popcll(m & lt);
            uint32_t old = 0;
            if (ok && below == 0) old = atomicAdd(&cnt[p], (uint32_t)__popcll(m));
            const uint32_t leader = m ? (uint32_t)(__ffsll((long long)m) - 1) : 0u;
            old = __shfl(old, (int)leader, kWave);
            rank[k] = old + below;
        } else {
            // the returned old value is the tuple's rank; lanes hitting the same
            // counter in one instruction get distinct values
            rank[k] = ok ? atomicAdd(&cnt[p], 1u) : 0u;
        }
    }
    const bool xok = (valid >> IPT) & 1u;
    const uint32_t xrank = xok ? atomicAdd(&cnt[part_of(kx, cfg)], 1u) : 0u;
    __syncthreads();
    uint32_t r_own = 0;  // counted: this thread's partition's reserved offset (in flight until used)
    // partitions of this tile whose HBM tables it clears (counted, P <= 64, R)
    uint64_t* s_clear = reinterpret_cast<uint64_t*>(ctot);  // (one word of the scan scratch)
    if (P <= kWave) {
        // One wave does it all (uniform branch): lane p scans the counts (local
        // starts) and, counted, the segment's totals (partition starts) and
        // reserves the tile's run; one barrier then publishes the starts.
        if (threadIdx.x < kWave) {
            const uint32_t p = threadIdx.x;
            const bool in = p < P;
            const uint32_t c = in ? cnt[p] : 0u;
            if (counted && in && c) r_own = atomicAdd(&rsv.cur[(uint64_t)t.seg * P + p], c);
            const uint32_t ec = wave_incl_scan(c) - c;
            const uint32_t g = in ? hs_own : 0u;
            const uint32_t base = counted ? wave_incl_scan(g) - g : g - seg0;  // start inside the segment
            if (in) {
                cnt[p] = ec;
                delta[p] = base - ec;  // counted: + r_own once it is back
            }
            // R partitions whose join takes an HBM table (counted: g is the partition's size)
            const uint64_t big = __ballot(in && rsv.ovf_table && t.seg < nseg / 2 && g > rsv.lds_cap);
            if (p == 0) *s_clear = big;
        }
        __syncthreads();
    } else if (counted) {
        // The segment's totals (the partition starts inside the segment, once
        // scanned) go to LDS first: a wait for their loads would also wait for
        // the reservations.  Then this tile's run of every partition is
        // reserved on the partition's cursor; the offsets are awaited only
        // after the scans and the reordering below.
        for (uint32_t p = threadIdx.x; p < Pp; p += BLOCK) delta[p] = p < P ? (p < BLOCK ? hs_own : hs[p]) : 0u;
        uint32_t* __restrict__ cur = rsv.cur + (uint64_t)t.seg * P;
        if (threadIdx.x < P) {
            const uint32_t c = cnt[threadIdx.x];
            r_own = c ? atomicAdd(&cur[threadIdx.x], c) : 0u;
        }
        for (uint32_t p = threadIdx.x + BLOCK; p < P; p += BLOCK) {
            const uint32_t c = cnt[p];
            resv[p] = c ? atomicAdd(&cur[p], c) : 0u;
        }
        __syncthreads();
        lds_excl_scan(cnt, Pp, ctot);
        __syncthreads();
        lds_excl_scan(delta, Pp, ctot);
        __syncthreads();
    } else {
        lds_excl_scan(cnt, Pp, ctot);
        __syncthreads();
        for (uint32_t p = threadIdx.x; p < P; p += BLOCK) {
            const uint32_t g = p < BLOCK ? hs_own : hs[(uint64_t)p * t.nt + t.tl];
            const uint32_t rel = g - seg0;  // exact: < segment length
            delta[p] = rel - cnt[p];
        }
    }
#pragma unroll
    for (uint32_t k = 0; k < IPT; ++k) {
        if ((valid >> k) & 1u) {
            const uint32_t pos = cnt[part_of(keys[k], cfg)] + rank[k];
            if (pos < T) {  // always true for consistent counts
                skey[pos] = keys[k];
                srid[pos] = rids[k];
            }
        }
    }
    if (xok) {
        const uint32_t pos = cnt[part_of(kx, cfg)] + xrank;
        if (pos < T) {
            skey[pos] = kx;
            srid[pos] = rx;
        }
    }
    // the reservations (and the prefetched offsets) are back by now; waiting
    // for them here keeps the waits out of the store loop below
    settle(r_own);
    settle(hs_own);
    if (counted) {  // global offset - local start
        if (P <= kWave) {
            if (threadIdx.x < P) delta[threadIdx.x] += r_own;
        } else {
            for (uint32_t p = threadIdx.x; p < P; p += BLOCK) delta[p] += (p < BLOCK ? r_own : resv[p]) - cnt[p];
        }
    }
    __syncthreads();
    int32_t* __restrict__ kout = key_out + sg.out_base;
    int32_t* __restrict__ rout = rid_out + sg.out_base;
    const uint64_t clear = (P <= kWave && rsv.ovf_table) ? *s_clear : 0ull;  // uniform
    if (clear == 0) {
#pragma unroll
        for (uint32_t k = 0; k < IPT; ++k) {
            const uint32_t j = k * BLOCK + threadIdx.x;
            if (j < t.len) {
                const int32_t key = skey[j];
                const uint32_t dst = delta[part_of(key, cfg)] + j;
                if (dst < sg.n) {  // always true for a consistent histogram scan; keeps stores in the segment
                    kout[dst] = key;
                    rout[dst] = srid[j];
                }
            }
        }
    } else {  // the same, and the 2 table slots of each tuple of a partition marked in `clear`
        uint4* __restrict__ slots = reinterpret_cast<uint4*>(rsv.ovf_table) + sg.out_base;  // R segment
#pragma unroll
        for (uint32_t k = 0; k < IPT; ++k) {
            const uint32_t j = k * BLOCK + threadIdx.x;
            if (j < t.len) {
                const int32_t key = skey[j];
                const uint32_t p = part_of(key, cfg);
                const uint32_t dst = delta[p] + j;
                if (dst < sg.n) {
                    kout[dst] = key;
                    rout[dst] = srid[j];
                    if ((clear >> p) & 1u) slots[dst] = make_uint4(~0u, ~0u, ~0u, ~0u);
                }
            }
        }
    }
}

// p1 != nullptr: pass 1 (tiles from *p1; grid >= 1 so the set-up always runs).
template <uint32_t BLOCK, uint32_t IPT>
void launch_hist(const PartSeg* segs, const uint32_t* tile_begin, const uint32_t* tile_seg, uint32_t nseg,
                 uint32_t grid, const PassCfg& cfg, uint32_t* hist, const Pass1* p1, Recorder& rec) {
    const bool count = p1 && p1->rows;
    if (count && (p1->bits_all < 4 || p1->bits_all > kCountedMaxBits)) {
        if (rec.err == hipSuccess) rec.err = hipErrorInvalidValue;
        return;
    }
    const size_t lds =
        sizeof(uint32_t) * (((size_t)1 << cfg.bits) + (count ? ((size_t)1 << p1->bits_all) + kCountEsc + 1 : 0));
    rec.before("part_hist");
    static_assert(BLOCK * IPT >= 1024 && BLOCK * IPT <= 8192 && BLOCK / kWave <= kScanScratch, "tile shape");
    if (count && cfg.nt)
        hipLaunchKernelGGL((k_part_hist<BLOCK, IPT, true, true, true>), dim3(grid), dim3(BLOCK), lds, rec.stream,
                           segs, tile_begin, tile_seg, nseg, cfg, hist, *p1);
    else if (count)
        hipLaunchKernelGGL((k_part_hist<BLOCK, IPT, true, true, false>), dim3(grid), dim3(BLOCK), lds, rec.stream,
                           segs, tile_begin, tile_seg, nseg, cfg, hist, *p1);
    else if (p1 && cfg.nt)
        hipLaunchKernelGGL((k_part_hist<BLOCK, IPT, true, false, true>), dim3(grid), dim3(BLOCK), lds, rec.stream,
                           segs, tile_begin, tile_seg, nseg, cfg, hist, *p1);
    else if (p1)
        hipLaunchKernelGGL((k_part_hist<BLOCK, IPT, true, false, false>), dim3(grid), dim3(BLOCK), lds, rec.stream,
                           segs, tile_begin, tile_seg, nseg, cfg, hist, *p1);
    else if (cfg.nt)
        hipLaunchKernelGGL((k_part_hist<BLOCK, IPT, false, false, true>), dim3(grid), dim3(BLOCK), lds, rec.stream,
                           segs, tile_begin, tile_seg, nseg, cfg, hist, Pass1{});
    else
        hipLaunchKernelGGL((k_part_hist<BLOCK, IPT, false, false, false>), dim3(grid), dim3(BLOCK), lds, rec.stream,
                           segs, tile_begin, tile_seg, nseg, cfg, hist, Pass1{});
    rec.after();
}

void hist_dispatch(const PartSeg* segs, const uint32_t* tile_begin, const uint32_t* tile_seg, uint32_t nseg,
                   uint32_t grid, const PassCfg& cfg, uint32_t* hist, const Pass1* p1, Recorder& rec) {
    // workgroup size by tile: part_block()
    switch (cfg.tile) {
        case 1024: launch_hist<256, 4>(segs, tile_begin, tile_seg, nseg, grid, cfg, hist, p1, rec); break;
        case 2048: launch_hist<256, 8>(segs, tile_begin, tile_seg, nseg, grid, cfg, hist, p1, rec); break;
        case 4096: launch_hist<512, 8>(segs, tile_begin, tile_seg, nseg, grid, cfg, hist, p1, rec); break;
        default: launch_hist<512, 16>(segs, tile_begin, tile_seg, nseg, grid, cfg, hist, p1, rec); break;
    }
}

template <uint32_t BLOCK, uint32_t IPT>
void launch_scatter(const PartSeg* segs, const uint32_t* tile_begin, const uint32_t* tile_seg, uint32_t nseg,
                    uint32_t grid, const PassCfg& cfg, const uint32_t* hist_scan, int32_t* key_out,
                    int32_t* rid_out, const SideJob& side, Recorder& rec, const Reserve& rsv) {
    if (part_block(cfg.tile) != BLOCK) {  // side-job workgroups are sized with part_block()
        if (rec.err == hipSuccess) rec.err = hipErrorInvalidConfiguration;
        return;
    }
    const size_t P = (size_t)1 << cfg.bits;
    const size_t Pp = P < kWave ? kWave : P;
    size_t lds = sizeof(uint32_t) * (2 * Pp + kScanScratch) + sizeof(int32_t) * 2 * BLOCK * IPT +
                 (rsv.tot && P > BLOCK ? sizeof(uint32_t) * Pp : 0);
    if (side.kind == kSideSetup2) {
        // room for the pass-2 segment tile offsets (else the setup fills the tile map from HBM)
        const size_t want = sizeof(uint32_t) * (kScanScratch + 2 * ((size_t)1 << side.setup2.bits1) + 1);
        if (want > lds && want <= 65536) lds = want;
    }
    const void* kern = cfg.nt ? (const void*)k_part_scatter<BLOCK, IPT, true>
                              : (const void*)k_part_scatter<BLOCK, IPT, false>;
    if (lds > 65536)
        (void)hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    rec.before("part_scatter");
    if (cfg.nt)
        hipLaunchKernelGGL((k_part_scatter<BLOCK, IPT, true>), dim3(side.front + grid + side.blocks), dim3(BLOCK),
                           lds, rec.stream, segs, tile_begin, tile_seg, nseg, cfg, hist_scan, key_out, rid_out, side,
                           (uint32_t)(lds / sizeof(uint32_t)), rsv);
    else
        hipLaunchKernelGGL((k_part_scatter<BLOCK, IPT, false>), dim3(side.front + grid + side.blocks), dim3(BLOCK),
                           lds, rec.stream, segs, tile_begin, tile_seg, nseg, cfg, hist_scan, key_out, rid_out, side,
                           (uint32_t)(lds / sizeof(uint32_t)), rsv);
    rec.after();
}

// starts[p] = first position of partition p in a one-segment pass (segment at
// output position 0, ntiles tiles, partition-major histogram scan), starts[P] = n.
__global__ void __launch_bounds__(256) k_part_starts(const uint32_t* __restrict__ hist_scan, uint32_t ntiles,
                                                    uint32_t P, uint32_t n, uint32_t* __restrict__ starts) {
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p <= P; p += gridDim.x * blockDim.x)
        starts[p] = (p == P || ntiles == 0) ? (p == P ? n : 0u) : min(hist_scan[(uint64_t)p * ntiles] - hist_scan[0], n);
}

}  // namespace

void part_starts(const uint32_t* hist_scan, uint32_t ntiles, uint32_t bits, uint32_t n, uint32_t* starts,
                 Recorder& rec) {
    const uint32_t P = 1u << bits;
    rec.before("part_starts");
    hipLaunchKernelGGL(k_part_starts, dim3((P + 256) / 256), dim3(256), 0, rec.stream, hist_scan, ntiles, P, n,
                       starts);
    rec.after();
}

size_t part_scatter_lds_bytes(uint32_t bits, uint32_t tile) {
    const size_t P = (size_t)1 << bits;
    const size_t Pp = P < kWave ? kWave : P;
    return sizeof(uint32_t) * (2 * Pp + kScanScratch) + sizeof(int32_t) * 2 * tile;
}

Pass1 make_pass1(const int32_t* rk, const int32_t* rr, uint32_t n_r, const int32_t* sk, const int32_t* sr,
                 uint32_t n_s, uint32_t tile, uint32_t bits, PartSeg* segs, uint32_t* tile_begin, uint64_t* zero,
                 uint64_t nzero, uint64_t* err_clear) {
    Pass1 a{};
    a.rk = rk;
    a.rr = rr;
    a.sk = sk;
    a.sr = sr;
    a.n_r = n_r;
    a.n_s = n_s;
    a.nt_r = (n_r + tile - 1) / tile;
    a.ntiles = a.nt_r + (n_s + tile - 1) / tile;
    a.hist_s = (uint64_t)a.nt_r << bits;
    a.segs = segs;
    a.tile_begin = tile_begin;
    a.zero = zero;
    a.nzero = nzero;
    a.err_clear = err_clear;
    return a;
}

void part_hist_pass1(const Pass1& p1, const PassCfg& cfg, uint32_t* hist, Recorder& rec) {
    hist_dispatch(p1.segs, p1.tile_begin, nullptr, 2, p1.ntiles ? p1.ntiles : 1u, cfg, hist, &p1, rec);
}

void part_hist(const PartSeg* segs, const uint32_t* tile_begin, const uint32_t* tile_seg, uint32_t nseg,
               uint32_t grid, const PassCfg& cfg, uint32_t* hist, Recorder& rec) {
    if (grid == 0) return;
    hist_dispatch(segs, tile_begin, tile_seg, nseg, grid, cfg, hist, nullptr, rec);
}

void part_scatter(const PartSeg* segs, const uint32_t* tile_begin, const uint32_t* tile_seg, uint32_t nseg,
                  uint32_t grid, const PassCfg& cfg, const uint32_t* hist_scan, int32_t* key_out,
                  int32_t* rid_out, const SideJob& side, Recorder& rec, const Reserve* rsv) {
    if (side.front + grid + side.blocks == 0) return;
    const Reserve r = rsv ? *rsv : Reserve{nullptr, nullptr, nullptr, 0u, 0u};
#define HJ_SCATTER(BLOCK, IPT) \
    launch_scatter<BLOCK, IPT>(segs, tile_begin, tile_seg, nseg, grid, cfg, hist_scan, key_out, rid_out, side, rec, r)
    switch (cfg.tile) {  // workgroup size by tile: part_block()
        case 1024: HJ_SCATTER(256, 4); break;
        case 2048: HJ_SCATTER(256, 8); break;
        case 4096: HJ_SCATTER(512, 8); break;
        default: HJ_SCATTER(512, 16); break;
    }
#undef HJ_SCATTER
}

}  // namespace hj
