// Join of the partition pairs of a PHJ ("apply SHJ on each partition pair",
// Algorithm 2; steps b1-b4 and p1-p4 of Algorithm 1 inside each pair).
//
// Work item = (partition pair i, chunk of kJoinChunk S tuples of S_i).  One
// workgroup per item:
//  * |R_i| <= lds_cap: R_i becomes a bucketed table in LDS.  The paper's
//    bucket header + key list + rid list (Section 3.1) is laid out without
//    pointers: bucket counts (LDS atomics, the latch of Section 3.3), an
//    in-LDS exclusive scan, then R_i's keys (and rids) placed bucket by bucket,
//    so bucket b is the contiguous run [end[b-1], end[b]).  Probing walks that
//    run (p3) and compares keys (p4).
//  * |R_i| > lds_cap (few, large partitions: low radix bits, duplicate-heavy
//    R): the pair is joined through a partition-local open-addressing table
//    in HBM (2 |R_i| slots at twice R_i's offset, plus per-key row chains),
//    built by separate clear/build launches with 64-bit compare-and-swap.
// Output: count pass -> per-wave counts -> scan -> write pass, which re-runs
// the same item and stores its pairs at the scanned offset (Section 3.3's
// dynamic output allocation replaced by counting).
#include "hj_device.h"
#include "hj_internal.h"

namespace hj {

namespace {

constexpr uint32_t kOvfChunk = 4096;                  // R tuples per HBM-table build item
constexpr uint32_t kSubJ = kJoinChunk / kJoinWaves;   // S tuples per wave of an item
constexpr uint32_t kPlanBlock = 1024;

__device__ __forceinline__ uint32_t floor_log2_min6(uint32_t n) {
    const uint32_t v = n < 64 ? 64u : n;
    return 31u - (uint32_t)__clz(v);
}

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

__global__ void __launch_bounds__(kPlanBlock) k_join_plan(
    const PartSeg* __restrict__ segs, const uint32_t* __restrict__ tile_begin, uint32_t nseg,
    uint32_t bits_last, const uint32_t* __restrict__ hist_scan, uint32_t n_r, uint32_t n_s,
    uint32_t total_bits, uint32_t lds_cap, PartPair* __restrict__ pairs,
    uint32_t* __restrict__ item_begin, uint32_t* __restrict__ ovf_begin) {
    __shared__ uint32_t wt[kPlanBlock / kWave];
    const uint32_t P = 1u << total_bits;
    const uint32_t nseg_rel = nseg / 2;
    const uint32_t per = (P + kPlanBlock - 1) / kPlanBlock;
    const uint32_t a = min(threadIdx.x * per, P);
    const uint32_t b = min(a + per, P);
    uint32_t items = 0, ovf = 0;
    uint32_t r0 = final_start(segs, tile_begin, hist_scan, 0, nseg_rel, bits_last, a, n_r, 0, P);
    uint32_t s0 = final_start(segs, tile_begin, hist_scan, 1, nseg_rel, bits_last, a, n_s, n_r, P);
    for (uint32_t i = a; i < b; ++i) {
        const uint32_t r1 = final_start(segs, tile_begin, hist_scan, 0, nseg_rel, bits_last, i + 1, n_r, 0, P);
        const uint32_t s1 = final_start(segs, tile_begin, hist_scan, 1, nseg_rel, bits_last, i + 1, n_s, n_r, P);
        PartPair pp;
        pp.r_off = r0; pp.r_len = r1 - r0; pp.s_off = s0; pp.s_len = s1 - s0;
        pairs[i] = pp;
        const bool live = pp.r_len && pp.s_len;
        items += live ? (pp.s_len + kJoinChunk - 1) / kJoinChunk : 0u;
        ovf += (live && pp.r_len > lds_cap) ? (pp.r_len + kOvfChunk - 1) / kOvfChunk : 0u;
        r0 = r1;
        s0 = s1;
    }
    uint32_t tot_items, tot_ovf;
    uint32_t run_i = block_excl_scan(items, wt, &tot_items);
    uint32_t run_o = block_excl_scan(ovf, wt, &tot_ovf);
    for (uint32_t i = a; i < b; ++i) {
        const PartPair pp = pairs[i];
        const bool live = pp.r_len && pp.s_len;
        item_begin[i] = run_i;
        ovf_begin[i] = run_o;
        run_i += live ? (pp.s_len + kJoinChunk - 1) / kJoinChunk : 0u;
        run_o += (live && pp.r_len > lds_cap) ? (pp.r_len + kOvfChunk - 1) / kOvfChunk : 0u;
    }
    if (threadIdx.x == 0) {
        item_begin[P] = tot_items;
        ovf_begin[P] = tot_ovf;
    }
}

__device__ __forceinline__ uint64_t region_slot(int32_t key, uint32_t H) {
    return ((uint64_t)slot_hash(key) * H) >> 32;
}

__global__ void __launch_bounds__(256) k_ovf_clear(const PartPair* __restrict__ pairs,
                                                  const uint32_t* __restrict__ ovf_begin, uint32_t P,
                                                  uint64_t* __restrict__ ovf_table) {
    const uint32_t item = blockIdx.x;
    if (item >= ovf_begin[P]) return;
    const uint32_t i = upper_index(ovf_begin, P, item);
    const uint32_t c = item - ovf_begin[i];
    const PartPair pp = pairs[i];
    uint64_t* region = ovf_table + 2ull * pp.r_off;
    const uint64_t H = 2ull * pp.r_len;
    const uint64_t end = min(2ull * (c + 1) * kOvfChunk, H);
    for (uint64_t x = 2ull * c * kOvfChunk + threadIdx.x; x < end; x += blockDim.x) region[x] = kEmptySlot;
}

struct RegionStep {
    uint32_t H;
    __device__ __forceinline__ uint64_t operator()(uint64_t s) const { return s + 1 == H ? 0 : s + 1; }
};

__global__ void __launch_bounds__(256) k_ovf_build(const PartPair* __restrict__ pairs,
                                                  const uint32_t* __restrict__ ovf_begin, uint32_t P,
                                                  const int32_t* __restrict__ rk,
                                                  uint64_t* __restrict__ ovf_table,
                                                  uint32_t* __restrict__ ovf_next) {
    const uint32_t item = blockIdx.x;
    if (item >= ovf_begin[P]) return;
    const uint32_t i = upper_index(ovf_begin, P, item);
    const uint32_t c = item - ovf_begin[i];
    const PartPair pp = pairs[i];
    uint64_t* region = ovf_table + 2ull * pp.r_off;
    uint32_t* next = ovf_next + pp.r_off;
    const RegionStep step{2u * pp.r_len};
    const uint32_t end = min((c + 1) * kOvfChunk, pp.r_len);
    for (uint32_t j = c * kOvfChunk + threadIdx.x; j < end; j += blockDim.x) {
        const int32_t k = rk[pp.r_off + j];
        chain_insert(region, next, region_slot(k, step.H), k, j, step);
    }
}

// Builds the bucketed LDS table over R_i: afterwards bucket b holds
// skey/srid[(b ? bend[b-1] : 0) .. bend[b]).  H = 2^log2H buckets.
template <bool kRids>
__device__ __forceinline__ void build_lds(const int32_t* __restrict__ rk, const int32_t* __restrict__ rr,
                                          uint32_t n, uint32_t log2H, uint32_t* bend, int32_t* skey,
                                          int32_t* srid, uint32_t* ctot) {
    const uint32_t H = 1u << log2H;
    const uint32_t sh = 32 - log2H;
    for (uint32_t x = threadIdx.x; x < H; x += blockDim.x) bend[x] = 0;
    __syncthreads();
    constexpr uint32_t U = 4;
    for (uint32_t base = 0; base < n; base += U * kJoinBlock) {
        int32_t k[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t j = base + u * kJoinBlock + threadIdx.x;
            k[u] = j < n ? rk[j] : 0;
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t j = base + u * kJoinBlock + threadIdx.x;
            if (j < n) atomicAdd(&bend[slot_hash(k[u]) >> sh], 1u);
        }
    }
    __syncthreads();
    lds_excl_scan(bend, H, ctot);
    __syncthreads();
    for (uint32_t base = 0; base < n; base += U * kJoinBlock) {
        int32_t k[U], r[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t j = base + u * kJoinBlock + threadIdx.x;
            k[u] = j < n ? rk[j] : 0;
            if (kRids) r[u] = j < n ? rr[j] : 0;
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t j = base + u * kJoinBlock + threadIdx.x;
            if (j < n) {
                const uint32_t pos = atomicAdd(&bend[slot_hash(k[u]) >> sh], 1u);
                skey[pos] = k[u];
                if (kRids) srid[pos] = r[u];
            }
        }
    }
    __syncthreads();
}

struct ItemLoc {
    uint32_t item;
    bool live;
    PartPair pp;
    uint32_t s_begin, s_n;
};

__device__ __forceinline__ ItemLoc locate_item(const PartPair* __restrict__ pairs,
                                               const uint32_t* __restrict__ item_begin, uint32_t P) {
    ItemLoc L;
    L.item = xcd_remap(blockIdx.x, gridDim.x);
    L.live = L.item < item_begin[P];
    if (!L.live) return L;
    const uint32_t i = upper_index(item_begin, P, L.item);
    const uint32_t c = L.item - item_begin[i];
    L.pp = pairs[i];
    L.s_begin = L.pp.s_off + c * kJoinChunk;
    L.s_n = min(kJoinChunk, L.pp.s_len - c * kJoinChunk);
    return L;
}

__global__ void __launch_bounds__(kJoinBlock) k_join_count(const PartPair* __restrict__ pairs,
                                                          const uint32_t* __restrict__ item_begin,
                                                          uint32_t P, const int32_t* __restrict__ rk,
                                                          const int32_t* __restrict__ sk, uint32_t lds_cap,
                                                          const uint64_t* __restrict__ ovf_table,
                                                          const uint32_t* __restrict__ ovf_next,
                                                          uint64_t* __restrict__ wave_cnt) {
    extern __shared__ uint32_t lds[];
    const uint32_t w = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const ItemLoc L = locate_item(pairs, item_begin, P);
    if (!L.live) {
        if (lane == 0) wave_cnt[(uint64_t)L.item * kJoinWaves + w] = 0;
        return;
    }
    uint64_t cnt = 0;
    const uint32_t wb = w * kSubJ;
    const uint32_t we = min(wb + kSubJ, L.s_n);
    const int32_t* __restrict__ skp = sk + L.s_begin;
    if (L.pp.r_len <= lds_cap) {
        uint32_t* bend = lds;
        int32_t* skey = (int32_t*)(lds + lds_cap);
        uint32_t* ctot = lds + 2 * lds_cap;
        const uint32_t log2H = floor_log2_min6(L.pp.r_len);
        build_lds<false>(rk + L.pp.r_off, nullptr, L.pp.r_len, log2H, bend, skey, nullptr, ctot);
        const uint32_t sh = 32 - log2H;
        for (uint32_t r = wb; r < we; r += kWave) {
            const uint32_t j = r + lane;
            if (j < we) {
                const int32_t k = skp[j];
                const uint32_t b = slot_hash(k) >> sh;
                const uint32_t lo = b ? bend[b - 1] : 0u;
                const uint32_t hi = bend[b];
                for (uint32_t x = lo; x < hi; ++x) cnt += (skey[x] == k);
            }
        }
    } else {
        const uint64_t* __restrict__ region = ovf_table + 2ull * L.pp.r_off;
        const uint32_t* __restrict__ next = ovf_next + L.pp.r_off;
        const RegionStep step{2u * L.pp.r_len};
        for (uint32_t r = wb; r < we; r += kWave) {
            const uint32_t j = r + lane;
            if (j < we) {
                const int32_t k = skp[j];
                const uint32_t h = chain_find(region, region_slot(k, step.H), k, step);
                if (h != kNotFound) cnt += chain_len(next, h);
            }
        }
    }
    cnt = wave_sum(cnt);
    if (lane == 0) wave_cnt[(uint64_t)L.item * kJoinWaves + w] = cnt;
}

__global__ void __launch_bounds__(kJoinBlock) k_join_write(
    const PartPair* __restrict__ pairs, const uint32_t* __restrict__ item_begin, uint32_t P,
    const int32_t* __restrict__ rk, const int32_t* __restrict__ rr, const int32_t* __restrict__ sk,
    const int32_t* __restrict__ sr, uint32_t lds_cap, const uint64_t* __restrict__ ovf_table,
    const uint32_t* __restrict__ ovf_next, const uint64_t* __restrict__ wave_base, int32_t* __restrict__ out_r, int32_t* __restrict__ out_s,
    uint64_t capacity) {
    extern __shared__ uint32_t lds[];
    const uint32_t w = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const ItemLoc L = locate_item(pairs, item_begin, P);
    if (!L.live) return;
    uint64_t pos0 = wave_base[(uint64_t)L.item * kJoinWaves + w];
    const uint32_t wb = w * kSubJ;
    const uint32_t we = min(wb + kSubJ, L.s_n);
    const int32_t* __restrict__ skp = sk + L.s_begin;
    const int32_t* __restrict__ srp = sr + L.s_begin;
    if (L.pp.r_len <= lds_cap) {
        uint32_t* bend = lds;
        int32_t* skey = (int32_t*)(lds + lds_cap);
        int32_t* srid = skey + lds_cap;
        uint32_t* ctot = (uint32_t*)(srid + lds_cap);
        const uint32_t log2H = floor_log2_min6(L.pp.r_len);
        build_lds<true>(rk + L.pp.r_off, rr + L.pp.r_off, L.pp.r_len, log2H, bend, skey, srid, ctot);
        const uint32_t sh = 32 - log2H;
        for (uint32_t r = wb; r < we; r += kWave) {
            const uint32_t j = r + lane;
            uint64_t c = 0;
            uint32_t lo = 0, hi = 0;
            int32_t k = 0;
            if (j < we) {
                k = skp[j];
                const uint32_t b = slot_hash(k) >> sh;
                lo = b ? bend[b - 1] : 0u;
                hi = bend[b];
                for (uint32_t x = lo; x < hi; ++x) c += (skey[x] == k);
            }
            const uint64_t incl = wave_incl_scan(c);
            uint64_t pos = pos0 + incl - c;
            pos0 += __shfl(incl, kWave - 1, kWave);
            if (c) {
                const int32_t rs = srp[j];
                for (uint32_t x = lo; x < hi; ++x) {
                    if (skey[x] == k) {
                        if (pos < capacity) {
                            out_r[pos] = srid[x];
                            out_s[pos] = rs;
                        }
                        ++pos;
                    }
                }
            }
        }
    } else {
        const uint64_t* __restrict__ region = ovf_table + 2ull * L.pp.r_off;
        const uint32_t* __restrict__ next = ovf_next + L.pp.r_off;
        const int32_t* __restrict__ rrp = rr + L.pp.r_off;
        const RegionStep step{2u * L.pp.r_len};
        for (uint32_t r = wb; r < we; r += kWave) {
            const uint32_t j = r + lane;
            uint64_t c = 0;
            uint32_t h = kNotFound;
            if (j < we) {
                const int32_t k = skp[j];
                h = chain_find(region, region_slot(k, step.H), k, step);
                if (h != kNotFound) c = chain_len(next, h);
            }
            const uint64_t incl = wave_incl_scan(c);
            uint64_t pos = pos0 + incl - c;
            pos0 += __shfl(incl, kWave - 1, kWave);
            if (c) {
                const int32_t rs = srp[j];
                while (true) {
                    const uint32_t row = h & ~kLast;
                    if (pos < capacity) {
                        out_r[pos] = rrp[row];
                        out_s[pos] = rs;
                    }
                    ++pos;
                    if (h & kLast) break;
                    h = next[row];
                }
            }
        }
    }
}

__global__ void k_write_zero(uint64_t* p) {
    if (threadIdx.x == 0) *p = 0;
}

}  // namespace

size_t join_lds_bytes(uint32_t lds_cap, bool write) {
    return sizeof(uint32_t) * ((size_t)lds_cap * (write ? 3 : 2) + lds_cap / kWave);
}

void write_zero_count(uint64_t* d_count, Recorder& rec) {
    rec.before("zero_count");
    hipLaunchKernelGGL(k_write_zero, dim3(1), dim3(64), 0, rec.stream, d_count);
    rec.after();
}

void join_plan(const PartSeg* segs, const uint32_t* tile_begin, uint32_t nseg, uint32_t bits_last,
               const uint32_t* hist_scan, uint32_t n_r, uint32_t n_s, uint32_t total_bits,
               uint32_t lds_cap, const JoinPlanOut& o, Recorder& rec) {
    rec.before("join_plan");
    hipLaunchKernelGGL(k_join_plan, dim3(1), dim3(kPlanBlock), 0, rec.stream, segs, tile_begin, nseg,
                       bits_last, hist_scan, n_r, n_s, total_bits, lds_cap, o.pairs, o.item_begin,
                       o.ovf_begin);
    rec.after();
}

uint32_t ovf_grid(uint32_t P, uint64_t n_r) {
    return (uint32_t)(P + (n_r + kOvfChunk - 1) / kOvfChunk);
}

uint32_t join_grid(uint32_t P, uint64_t n_s) {
    return (uint32_t)(P + (n_s + kJoinChunk - 1) / kJoinChunk);
}

void join_ovf_build(const PartPair* pairs, const uint32_t* ovf_begin, uint32_t P, uint32_t grid,
                    const int32_t* rk, uint64_t* ovf_table, uint32_t* ovf_next, Recorder& rec) {
    if (grid == 0) return;
    rec.before("ovf_clear");
    hipLaunchKernelGGL(k_ovf_clear, dim3(grid), dim3(256), 0, rec.stream, pairs, ovf_begin, P, ovf_table);
    rec.after();
    rec.before("ovf_build");
    hipLaunchKernelGGL(k_ovf_build, dim3(grid), dim3(256), 0, rec.stream, pairs, ovf_begin, P, rk,
                       ovf_table, ovf_next);
    rec.after();
}

void join_count(const PartPair* pairs, const uint32_t* item_begin, uint32_t P, uint32_t grid,
                const int32_t* rk, const int32_t* sk, uint32_t lds_cap, const uint64_t* ovf_table,
                const uint32_t* ovf_next, uint64_t* wave_cnt, Recorder& rec) {
    if (grid == 0) return;
    const size_t lds = join_lds_bytes(lds_cap, false);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void*)k_join_count, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
    rec.before("join_count");
    hipLaunchKernelGGL(k_join_count, dim3(grid), dim3(kJoinBlock), lds, rec.stream, pairs, item_begin, P,
                       rk, sk, lds_cap, ovf_table, ovf_next, wave_cnt);
    rec.after();
}

void join_write(const PartPair* pairs, const uint32_t* item_begin, uint32_t P, uint32_t grid,
                const int32_t* rk, const int32_t* rr, const int32_t* sk, const int32_t* sr,
                uint32_t lds_cap, const uint64_t* ovf_table, const uint32_t* ovf_next,
                const uint64_t* wave_base, int32_t* out_r, int32_t* out_s, uint64_t capacity,
                Recorder& rec) {
    if (grid == 0) return;
    const size_t lds = join_lds_bytes(lds_cap, true);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void*)k_join_write, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
    rec.before("join_write");
    hipLaunchKernelGGL(k_join_write, dim3(grid), dim3(kJoinBlock), lds, rec.stream, pairs, item_begin, P,
                       rk, rr, sk, sr, lds_cap, ovf_table, ovf_next, wave_base, out_r, out_s, capacity);
    rec.after();
}

}  // namespace hj
