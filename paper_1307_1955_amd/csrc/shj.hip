// Simple hash join (SHJ), Algorithm 1 (Section 3.1), on one device-wide table.
//
// The paper's table -- bucket headers, a key list per bucket, a rid list per
// key (Section 3.1) -- needs dynamic allocation inside the kernel (Section
// 3.3).  Here it is an array of 2^L 64-bit slots, L = ceil(log2(2 |R|)), plus
// one uint32 `next` per R row:
//   * a slot is one distinct key and the head of its row chain (the key node
//     and its rid list); linear probing over slots plays the bucket's key list;
//   * next[row] links the rows of a duplicated key (the rid list), so
//     duplicates cost one push each instead of lengthening probe sequences.
// build  b1: slot = mix(key); b2/b3: probe to the key's slot or claim an empty
//        one with a 64-bit compare-and-swap (the latch of Section 3.3 becomes
//        one HBM atomic per tuple); b4: push the row onto the key's chain.
// probe  p1-p3: probe to the key's slot or the first empty slot; p4: every
//        row of the chain is one output pair.
// Output is materialised in two passes (count -> scan -> write), so nothing is
// allocated on the device and the result lands contiguously.
#include "hj_device.h"
#include "hj_heavy.h"
#include "hj_internal.h"

namespace hj {

namespace {

__global__ void __launch_bounds__(256) k_fill_u64(uint64_t* __restrict__ p, uint64_t n, uint64_t v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 2;
    for (uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2; i < n; i += stride) {
        if (i + 1 < n) {
            *reinterpret_cast<ulonglong2*>(p + i) = make_ulonglong2(v, v);
        } else {
            p[i] = v;
        }
    }
}

struct PowStep {
    uint64_t mask;
    __device__ __forceinline__ uint64_t operator()(uint64_t s) const { return (s + 1) & mask; }
};

__device__ __forceinline__ uint64_t home_slot(int32_t k, uint32_t log2_slots) {
    return (uint64_t)(slot_hash(k) >> (32 - log2_slots));
}

__global__ void __launch_bounds__(256) k_shj_build(const int32_t* __restrict__ key, uint64_t n,
                                                  uint64_t* __restrict__ table, uint32_t* __restrict__ next,
                                                  uint32_t log2_slots) {
    constexpr uint32_t kWaves = 256 / kWave;
    __shared__ WavePush::Run runs[kWaves];
    const PowStep step{(1ull << log2_slots) - 1};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    WavePush push;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x; i0 < n; i0 += stride) {  // uniform trip count
        const uint64_t i = i0 + threadIdx.x;
        int32_t k = 0;
        uint64_t s = kClaimed;
        if (i < n) {
            k = key[i];
            s = push.hot(k) ? push.hot_slot : chain_claim(table, home_slot(k, log2_slots), k, (uint32_t)i, step);
        }
        push.add(table, next, s, k, (uint32_t)i);
    }
    push.flush_block<kWaves>(table, next, runs);
}

// Probe tiles: tile t covers S rows [t*kShjTile, ...); wave w of the block takes
// the contiguous range [w*kSub, (w+1)*kSub) of it; lane l handles rows
// u*64 + l, one round per u.  (Issuing all kSU first reads together was
// measured slower on MI355X: the random reads into a table far larger than
// the caches are bound by line fetches, not by latency.)
constexpr uint32_t kSub = kShjTile / kShjWavesPerBlock;
constexpr uint32_t kSU = kSub / kWave;

// An S tuple whose chain is longer than heavy_limit(|R|) is registered in hs
// and counted and written by the whole block (cooperative scan of R).
// hs->n must be zero and visible to the block before the call.
template <bool kRids>
__device__ __forceinline__ void shj_probe(const int32_t* __restrict__ s_key, const int32_t* __restrict__ s_rid,
                                          uint64_t begin, uint64_t n_s, const uint64_t* __restrict__ table,
                                          const uint32_t* __restrict__ next, uint32_t log2_slots, uint32_t lim,
                                          HeavySet* hs, int32_t* q, int32_t* qr, uint32_t* head, uint32_t* cnt) {
    const PowStep step{(1ull << log2_slots) - 1};
#pragma unroll
    for (uint32_t u = 0; u < kSU; ++u) {
        const uint64_t j = begin + u * kWave + lane_id();
        head[u] = kNotFound;
        cnt[u] = 0;
        q[u] = 0;
        if (kRids) qr[u] = 0;
        if (j < n_s) {
            q[u] = s_key[j];
            if (kRids) qr[u] = s_rid[j];
            head[u] = chain_find(table, home_slot(q[u], log2_slots), q[u], step);
            if (head[u] != kNotFound) cnt[u] = heavy_or_len(next, head[u], lim, q[u], kRids ? qr[u] : 0, hs);
        }
    }
}

__device__ __forceinline__ uint32_t count_of(uint32_t c, const HeavySet* hs) {
    return is_heavy(c) ? hs->cnt[c & ~kHeavyBit] : c;
}

__global__ void __launch_bounds__(kShjBlock) k_shj_count(const int32_t* __restrict__ s_key, uint64_t n_s,
                                                        const uint64_t* __restrict__ table,
                                                        const uint32_t* __restrict__ next,
                                                        uint32_t log2_slots, const int32_t* __restrict__ r_key,
                                                        uint64_t n_r, uint64_t* __restrict__ wave_cnt) {
    __shared__ HeavySet hs;
    const uint32_t w = threadIdx.x / kWave;
    const uint64_t begin = (uint64_t)blockIdx.x * kShjTile + (uint64_t)w * kSub;
    if (threadIdx.x == 0) hs.n = 0;
    __syncthreads();
    int32_t q[kSU], qr[kSU];
    uint32_t head[kSU], c[kSU];
    shj_probe<false>(s_key, nullptr, begin, n_s, table, next, log2_slots, heavy_limit(n_r), &hs, q, qr, head, c);
    heavy_counts<kShjBlock, kHeavyV>(r_key, n_r, &hs);
    uint64_t cnt = 0;
#pragma unroll
    for (uint32_t u = 0; u < kSU; ++u) cnt += count_of(c[u], &hs);
    cnt = wave_sum(cnt);
    if (lane_id() == 0) wave_cnt[(uint64_t)blockIdx.x * kShjWavesPerBlock + w] = cnt;
}

// Write pass; kOnePass reserves the block's output with one atomic add on the
// running total instead of reading a scanned offset (see HJ_FLAG_ONE_PASS).
template <bool kOnePass>
__global__ void __launch_bounds__(kShjBlock) k_shj_write(
    const int32_t* __restrict__ s_key, const int32_t* __restrict__ s_rid, uint64_t n_s,
    const uint64_t* __restrict__ table, const uint32_t* __restrict__ next, uint32_t log2_slots,
    const int32_t* __restrict__ r_key, const int32_t* __restrict__ r_rid, uint64_t n_r,
    const uint64_t* __restrict__ wave_base, unsigned long long* __restrict__ total, int32_t* __restrict__ out_r,
    int32_t* __restrict__ out_s, uint64_t capacity) {
    __shared__ uint64_t wtot[kShjWavesPerBlock + 1];
    __shared__ HeavySet hs;
    const uint32_t w = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const uint64_t begin = (uint64_t)blockIdx.x * kShjTile + (uint64_t)w * kSub;
    if (threadIdx.x == 0) hs.n = 0;
    __syncthreads();
    int32_t q[kSU], qr[kSU];
    uint32_t head[kSU], c[kSU];
    shj_probe<true>(s_key, s_rid, begin, n_s, table, next, log2_slots, heavy_limit(n_r), &hs, q, qr, head, c);
    heavy_counts<kShjBlock, kHeavyV>(r_key, n_r, &hs);
    uint64_t pos0;
    if (kOnePass) {
        uint64_t mine = 0;
#pragma unroll
        for (uint32_t u = 0; u < kSU; ++u) mine += count_of(c[u], &hs);
        mine = wave_sum(mine);
        if (lane == 0) wtot[w] = mine;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t t = 0;
            for (uint32_t i = 0; i < kShjWavesPerBlock; ++i) t += wtot[i];
            wtot[kShjWavesPerBlock] = t ? atomicAdd(total, (unsigned long long)t) : 0ull;
        }
        __syncthreads();
        pos0 = wtot[kShjWavesPerBlock];
        for (uint32_t i = 0; i < w; ++i) pos0 += wtot[i];
    } else {
        pos0 = wave_base[(uint64_t)blockIdx.x * kShjWavesPerBlock + w];
    }
#pragma unroll
    for (uint32_t u = 0; u < kSU; ++u) {
        const uint32_t cu = count_of(c[u], &hs);
        uint64_t excl, wtotal;
        wave_offsets(cu, &excl, &wtotal);
        uint64_t pos = pos0 + excl;
        pos0 += wtotal;
        if (is_heavy(c[u])) {
            hs.pos[c[u] & ~kHeavyBit] = pos;
        } else if (cu) {
            uint32_t h = head[u];
            while (true) {
                const uint32_t row = h & ~kLast;
                if (pos < capacity) {
                    out_r[pos] = r_rid[row];
                    out_s[pos] = qr[u];
                }
                ++pos;
                if (h & kLast) break;
                h = next[row];
            }
        }
    }
    heavy_writes<kShjBlock, kHeavyV>(r_key, r_rid, n_r, &hs, capacity, out_r, out_s);
}

__global__ void k_zero_u64(uint64_t* p) {
    if (threadIdx.x == 0) *p = 0;
}

}  // namespace

void shj_fill(uint64_t* table, uint64_t nslots, uint64_t* zero_total, Recorder& rec) {
    uint64_t blocks = (nslots / 2 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    rec.before("shj_fill");
    hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)blocks), dim3(256), 0, rec.stream, table, nslots,
                       kEmptySlot);
    rec.after();
    if (zero_total) {
        rec.before("zero_count");
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, rec.stream, zero_total);
        rec.after();
    }
}

void shj_build(const int32_t* key, uint64_t n, uint64_t* table, uint32_t* next, uint32_t log2_slots,
               Recorder& rec) {
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;  // grid-stride: a wave's pending push chain spans its rows
    if (blocks == 0) return;
    rec.before("shj_build");
    hipLaunchKernelGGL(k_shj_build, dim3((uint32_t)blocks), dim3(256), 0, rec.stream, key, n, table, next,
                       log2_slots);
    rec.after();
}

void shj_count(const int32_t* s_key, uint64_t n_s, const uint64_t* table, const uint32_t* next,
               uint32_t log2_slots, const int32_t* r_key, uint64_t n_r, uint64_t* wave_cnt, Recorder& rec) {
    const uint64_t tiles = (n_s + kShjTile - 1) / kShjTile;
    if (tiles == 0) return;
    rec.before("shj_count");
    hipLaunchKernelGGL(k_shj_count, dim3((uint32_t)tiles), dim3(kShjBlock), 0, rec.stream, s_key, n_s,
                       table, next, log2_slots, r_key, n_r, wave_cnt);
    rec.after();
}

void shj_write(const int32_t* s_key, const int32_t* s_rid, uint64_t n_s, const uint64_t* table,
               const uint32_t* next, uint32_t log2_slots, const int32_t* r_key, const int32_t* r_rid,
               uint64_t n_r, const uint64_t* wave_base, uint64_t* total, int32_t* out_r, int32_t* out_s,
               uint64_t capacity, Recorder& rec) {
    const uint64_t tiles = (n_s + kShjTile - 1) / kShjTile;
    if (tiles == 0) return;
    if (wave_base == nullptr) {
        rec.before("shj_write_1pass");
        hipLaunchKernelGGL(k_shj_write<true>, dim3((uint32_t)tiles), dim3(kShjBlock), 0, rec.stream, s_key,
                           s_rid, n_s, table, next, log2_slots, r_key, r_rid, n_r, wave_base, (unsigned long long*)total,
                           out_r, out_s, capacity);
    } else {
        rec.before("shj_write");
        hipLaunchKernelGGL(k_shj_write<false>, dim3((uint32_t)tiles), dim3(kShjBlock), 0, rec.stream, s_key,
                           s_rid, n_s, table, next, log2_slots, r_key, r_rid, n_r, wave_base, (unsigned long long*)total,
                           out_r, out_s, capacity);
    }
    rec.after();
}

}  // namespace hj
