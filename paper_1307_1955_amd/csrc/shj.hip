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
    const PowStep step{(1ull << log2_slots) - 1};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t k = key[i];
        chain_insert(table, next, home_slot(k, log2_slots), k, (uint32_t)i, step);
    }
}

// Probe tiles: tile t covers S rows [t*kShjTile, ...); wave w of the block takes
// the contiguous range [w*kSub, (w+1)*kSub) of it, 64 rows per round.
constexpr uint32_t kSub = kShjTile / kShjWavesPerBlock;

__global__ void __launch_bounds__(kShjBlock) k_shj_count(const int32_t* __restrict__ s_key, uint64_t n_s,
                                                        const uint64_t* __restrict__ table,
                                                        const uint32_t* __restrict__ next,
                                                        uint32_t log2_slots,
                                                        uint64_t* __restrict__ wave_cnt) {
    const PowStep step{(1ull << log2_slots) - 1};
    const uint32_t w = threadIdx.x / kWave;
    const uint64_t begin = (uint64_t)blockIdx.x * kShjTile + (uint64_t)w * kSub;
    uint64_t cnt = 0;
    for (uint32_t r = 0; r < kSub; r += kWave) {
        const uint64_t j = begin + r + lane_id();
        if (j < n_s) {
            const int32_t k = s_key[j];
            const uint32_t h = chain_find(table, home_slot(k, log2_slots), k, step);
            if (h != kNotFound) cnt += chain_len(next, h);
        }
    }
    cnt = wave_sum(cnt);
    if (lane_id() == 0) wave_cnt[(uint64_t)blockIdx.x * kShjWavesPerBlock + w] = cnt;
}

__global__ void __launch_bounds__(kShjBlock) k_shj_write(
    const int32_t* __restrict__ s_key, const int32_t* __restrict__ s_rid, uint64_t n_s,
    const uint64_t* __restrict__ table, const uint32_t* __restrict__ next, uint32_t log2_slots,
    const int32_t* __restrict__ r_rid, const uint64_t* __restrict__ wave_base,
    int32_t* __restrict__ out_r, int32_t* __restrict__ out_s, uint64_t capacity) {
    const PowStep step{(1ull << log2_slots) - 1};
    const uint32_t w = threadIdx.x / kWave;
    const uint64_t begin = (uint64_t)blockIdx.x * kShjTile + (uint64_t)w * kSub;
    uint64_t pos0 = wave_base[(uint64_t)blockIdx.x * kShjWavesPerBlock + w];
    for (uint32_t r = 0; r < kSub; r += kWave) {
        const uint64_t j = begin + r + lane_id();
        uint64_t c = 0;
        uint32_t h = kNotFound;
        if (j < n_s) {
            const int32_t k = s_key[j];
            h = chain_find(table, home_slot(k, log2_slots), k, step);
            if (h != kNotFound) c = chain_len(next, h);
        }
        const uint64_t incl = wave_incl_scan(c);
        uint64_t pos = pos0 + incl - c;
        pos0 += __shfl(incl, kWave - 1, kWave);
        if (c) {
            const int32_t sr = s_rid[j];
            while (true) {
                const uint32_t row = h & ~kLast;
                if (pos < capacity) {
                    out_r[pos] = r_rid[row];
                    out_s[pos] = sr;
                }
                ++pos;
                if (h & kLast) break;
                h = next[row];
            }
        }
    }
}

}  // namespace

void shj_fill(uint64_t* table, uint64_t nslots, Recorder& rec) {
    uint64_t blocks = (nslots / 2 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    rec.before("shj_fill");
    hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)blocks), dim3(256), 0, rec.stream, table, nslots,
                       kEmptySlot);
    rec.after();
}

void shj_build(const int32_t* key, uint64_t n, uint64_t* table, uint32_t* next, uint32_t log2_slots,
               Recorder& rec) {
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks == 0) return;
    rec.before("shj_build");
    hipLaunchKernelGGL(k_shj_build, dim3((uint32_t)blocks), dim3(256), 0, rec.stream, key, n, table, next,
                       log2_slots);
    rec.after();
}

void shj_count(const int32_t* s_key, uint64_t n_s, const uint64_t* table, const uint32_t* next,
               uint32_t log2_slots, uint64_t* wave_cnt, Recorder& rec) {
    const uint64_t tiles = (n_s + kShjTile - 1) / kShjTile;
    if (tiles == 0) return;
    rec.before("shj_count");
    hipLaunchKernelGGL(k_shj_count, dim3((uint32_t)tiles), dim3(kShjBlock), 0, rec.stream, s_key, n_s,
                       table, next, log2_slots, wave_cnt);
    rec.after();
}

void shj_write(const int32_t* s_key, const int32_t* s_rid, uint64_t n_s, const uint64_t* table,
               const uint32_t* next, uint32_t log2_slots, const int32_t* r_rid,
               const uint64_t* wave_base, int32_t* out_r, int32_t* out_s, uint64_t capacity,
               Recorder& rec) {
    const uint64_t tiles = (n_s + kShjTile - 1) / kShjTile;
    if (tiles == 0) return;
    rec.before("shj_write");
    hipLaunchKernelGGL(k_shj_write, dim3((uint32_t)tiles), dim3(kShjBlock), 0, rec.stream, s_key, s_rid,
                       n_s, table, next, log2_slots, r_rid, wave_base, out_r, out_s, capacity);
    rec.after();
}

}  // namespace hj
