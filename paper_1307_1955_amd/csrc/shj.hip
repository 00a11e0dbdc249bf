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
//        one HBM atomic per new key); b4: push the row onto the key's chain
//        (exchange pushes, joined per wave and per workgroup; WavePush).
// probe  p1-p3: probe to the key's slot or the first empty slot; p4: every
//        row of the chain is one output pair.  Tuples on very long chains are
//        handled by whole workgroups (below, and hj_heavy.h).
// Output is materialised in two passes (count -> scan -> write) or in one
// (block reservation on a running total); nothing is allocated on the device
// and the result lands contiguously.
#include "hj_device.h"
#include "hj_heavy.h"
#include "hj_internal.h"

namespace hj {

namespace {

__global__ void __launch_bounds__(256) k_fill_u64(uint64_t* __restrict__ p, uint64_t n, uint64_t v,
                                                 uint32_t* __restrict__ zero, uint32_t zero_words,
                                                 uint64_t* __restrict__ err_clear) {
    if (blockIdx.x == 0) {
        for (uint32_t i = threadIdx.x; i < zero_words; i += blockDim.x) zero[i] = 0;
        if (threadIdx.x == 0 && err_clear) *err_clear = 0;
    }
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 2;
    for (uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2; i < n; i += stride) {
        if (i + 1 < n) {
            *reinterpret_cast<ulonglong2*>(p + i) = make_ulonglong2(v, v);
        } else {
            p[i] = v;
        }
    }
}

// Linear probing over nslots slots (any count: the home slot comes from a
// multiply-shift of the key's mix, so the table can be sized to the caches).
struct WrapStep {
    uint64_t nslots;
    __device__ __forceinline__ uint64_t operator()(uint64_t s) const { return s + 1 == nslots ? 0 : s + 1; }
};

__device__ __forceinline__ uint64_t home_slot(int32_t k, uint64_t nslots) {
    return ((uint64_t)slot_hash(k) * nslots) >> 32;
}

template <bool kNt>
__global__ void __launch_bounds__(256) k_shj_build(const int32_t* __restrict__ key, uint64_t n,
                                                  uint64_t* __restrict__ table, uint32_t* __restrict__ next,
                                                  uint64_t nslots, HotKeys* hot) {
    constexpr uint32_t kWaves = 256 / kWave;
    __shared__ WavePush::Run runs[kWaves];
    const WrapStep step{nslots};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    WavePush push;
    push.hot_keys = hot;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x; i0 < n; i0 += stride) {  // uniform trip count
        const uint64_t i = i0 + threadIdx.x;
        int32_t k = 0;
        uint64_t s = kClaimed;
        if (i < n) {
            k = kNt ? __builtin_nontemporal_load(key + i) : key[i];  // read once
            s = push.hot(k) ? push.hot_slot : chain_claim(table, home_slot(k, nslots), k, (uint32_t)i, step);
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

// An S tuple whose chain is longer than lim is registered in hs as heavy.  When
// the build recorded its key as hot (hk[0..nhk), LDS) with more than lim rows
// (hr: the recorded lower bound of the chain length), it is registered without
// walking the chain; otherwise the walk decides.
// hs->n must be zero and visible to the block before the call.
template <bool kRids>
__device__ __forceinline__ void shj_probe(const int32_t* __restrict__ s_key, const int32_t* __restrict__ s_rid,
                                          uint64_t begin, uint64_t n_s, const uint64_t* __restrict__ table,
                                          const uint32_t* __restrict__ next, uint64_t nslots, uint32_t lim,
                                          const int32_t* hk, const uint32_t* hr, uint32_t nhk, HeavySet* hs,
                                          int32_t* q, int32_t* qr,
                                          uint32_t* head, uint32_t* cnt) {
    const WrapStep step{nslots};
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
            head[u] = chain_find(table, home_slot(q[u], nslots), q[u], step);
            if (head[u] != kNotFound) {
                // a chain of one row is never heavy
                const uint32_t hot_rows = (head[u] & kLast) ? 0u : hot_rows_of(q[u], hk, hr, nhk);
                cnt[u] = hot_rows > lim ? register_heavy(next, head[u], q[u], kRids ? qr[u] : 0, hs)
                                        : heavy_or_len(next, head[u], lim, q[u], kRids ? qr[u] : 0, hs);
            }
        }
    }
}

__device__ __forceinline__ uint32_t count_of(uint32_t c, const HeavySet* hs) {
    return is_heavy(c) ? hs->cnt[c & ~kHeavyBit] : c;
}

__global__ void __launch_bounds__(kShjBlock) k_shj_count(const int32_t* __restrict__ s_key, uint64_t n_s,
                                                        const uint64_t* __restrict__ table,
                                                        const uint32_t* __restrict__ next,
                                                        uint64_t nslots, const int32_t* __restrict__ r_key,
                                                        uint64_t n_r, const HotKeys* __restrict__ hot,
                                                        uint64_t* __restrict__ wave_cnt,
                                                        uint64_t* __restrict__ err_clear) {
    __shared__ HeavySet hs;
    if (blockIdx.x == 0 && threadIdx.x == 0 && err_clear) *err_clear = 0;
    __shared__ int32_t hk[kHotKeys];
    __shared__ uint32_t hr[kHotKeys];
    __shared__ uint32_t nhk;
    const uint32_t w = threadIdx.x / kWave;
    const uint64_t begin = (uint64_t)blockIdx.x * kShjTile + (uint64_t)w * kSub;
    load_hot(hot, hk, hr, &nhk);
    if (threadIdx.x == 0) hs.n = hs.queued = 0;
    __syncthreads();
    int32_t q[kSU], qr[kSU];
    uint32_t head[kSU], c[kSU];
    shj_probe<false>(s_key, nullptr, begin, n_s, table, next, nslots, heavy_limit(n_r), hk, hr, nhk, &hs, q, qr,
                     head, c);
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
__global__ void __launch_bounds__(kShjBlock) __attribute__((amdgpu_waves_per_eu(8))) k_shj_write(
    const int32_t* __restrict__ s_key, const int32_t* __restrict__ s_rid, uint64_t n_s,
    const uint64_t* __restrict__ table, const uint32_t* __restrict__ next, uint64_t nslots,
    const int32_t* __restrict__ r_key, const int32_t* __restrict__ r_rid, uint64_t n_r,
    const HotKeys* __restrict__ hot, const uint64_t* __restrict__ wave_base,
    unsigned long long* __restrict__ total, HeavyQueue* heavy, int32_t* __restrict__ out_r,
    int32_t* __restrict__ out_s, uint64_t capacity) {
    __shared__ uint64_t wtot[kShjWavesPerBlock + 1];
    __shared__ HeavySet hs;
    __shared__ int32_t hk[kHotKeys];
    __shared__ uint32_t hr[kHotKeys];
    __shared__ uint32_t nhk;
    const uint32_t w = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const uint64_t begin = (uint64_t)blockIdx.x * kShjTile + (uint64_t)w * kSub;
    load_hot(hot, hk, hr, &nhk);
    if (threadIdx.x == 0) hs.n = hs.queued = 0;
    __syncthreads();
    int32_t q[kSU], qr[kSU];
    uint32_t head[kSU], c[kSU];
    // one-pass: a chain is heavy from kQueueWalk rows on (handed to every workgroup)
    const uint32_t lim = kOnePass ? min(heavy_limit(n_r), kQueueWalk) : heavy_limit(n_r);
    shj_probe<true>(s_key, s_rid, begin, n_s, table, next, nslots, lim, hk, hr, nhk, &hs, q, qr, head, c);
    // with R in one chunk the queue adds no workgroups to a tuple: keep the block's own scan
    if (kOnePass && n_r > kHelpChunk) hand_off(heavy, &hs, 0u, (uint32_t)n_r);
    heavy_counts<kShjBlock, kHeavyV, kOnePass>(r_key, n_r, &hs);
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
    heavy_writes<kShjBlock, kHeavyV, true>(r_key, r_rid, n_r, &hs, capacity, out_r, out_s);
    if (kOnePass) help_heavy<kShjBlock>(heavy, r_key, r_rid, total, capacity, out_r, out_s, hs.wsum);
}

__global__ void __launch_bounds__(256) k_zero_one_pass(uint64_t* __restrict__ total, uint64_t* __restrict__ q,
                                                      uint64_t* __restrict__ err_clear) {
    if (threadIdx.x == 0) {
        *total = 0;
        if (err_clear) *err_clear = 0;
    }
    for (uint32_t i = threadIdx.x; i < sizeof(HeavyQueue) / 8; i += blockDim.x) q[i] = 0;
}

}  // namespace

void shj_fill(uint64_t* table, uint64_t nslots, HotKeys* hot, Recorder& rec) {
    uint64_t blocks = (nslots / 2 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    rec.before("shj_fill");
    hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)blocks), dim3(256), 0, rec.stream, table, nslots,
                       kEmptySlot, reinterpret_cast<uint32_t*>(hot), (uint32_t)(sizeof(HotKeys) / 4), rec.err_clear);
    rec.after();
}

void shj_zero_one_pass(uint64_t* d_count, HeavyQueue* q, Recorder& rec) {
    rec.before("zero_count");
    hipLaunchKernelGGL(k_zero_one_pass, dim3(1), dim3(256), 0, rec.stream, d_count, reinterpret_cast<uint64_t*>(q),
                       rec.err_clear);
    rec.after();
}

void shj_build(const int32_t* key, uint64_t n, uint64_t* table, uint32_t* next, uint64_t nslots,
               HotKeys* hot, bool nt, Recorder& rec) {
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;  // grid-stride: a wave's pending push chain spans its rows
    if (blocks == 0) return;
    rec.before("shj_build");
    if (nt)
        hipLaunchKernelGGL(k_shj_build<true>, dim3((uint32_t)blocks), dim3(256), 0, rec.stream, key, n, table,
                           next, nslots, hot);
    else
        hipLaunchKernelGGL(k_shj_build<false>, dim3((uint32_t)blocks), dim3(256), 0, rec.stream, key, n, table,
                           next, nslots, hot);
    rec.after();
}

void shj_count(const int32_t* s_key, uint64_t n_s, const uint64_t* table, const uint32_t* next,
               uint64_t nslots, const int32_t* r_key, uint64_t n_r, const HotKeys* hot, uint64_t* wave_cnt,
               Recorder& rec) {
    const uint64_t tiles = (n_s + kShjTile - 1) / kShjTile;
    if (tiles == 0) return;
    rec.before("shj_count");
    hipLaunchKernelGGL(k_shj_count, dim3((uint32_t)tiles), dim3(kShjBlock), 0, rec.stream, s_key, n_s,
                       table, next, nslots, r_key, n_r, hot, wave_cnt, rec.err_clear);
    rec.after();
}

void shj_write(const int32_t* s_key, const int32_t* s_rid, uint64_t n_s, const uint64_t* table,
               const uint32_t* next, uint64_t nslots, const int32_t* r_key, const int32_t* r_rid,
               uint64_t n_r, const HotKeys* hot, const uint64_t* wave_base, uint64_t* total, HeavyQueue* heavy,
               int32_t* out_r, int32_t* out_s, uint64_t capacity, Recorder& rec) {
    const uint64_t tiles = (n_s + kShjTile - 1) / kShjTile;
    if (tiles == 0) return;
    if (wave_base == nullptr) {
        rec.before("shj_write_1pass");
        hipLaunchKernelGGL(k_shj_write<true>, dim3((uint32_t)tiles), dim3(kShjBlock), 0, rec.stream, s_key,
                           s_rid, n_s, table, next, nslots, r_key, r_rid, n_r, hot, wave_base,
                           (unsigned long long*)total, heavy, out_r, out_s, capacity);
    } else {
        rec.before("shj_write");
        hipLaunchKernelGGL(k_shj_write<false>, dim3((uint32_t)tiles), dim3(kShjBlock), 0, rec.stream, s_key,
                           s_rid, n_s, table, next, nslots, r_key, r_rid, n_r, hot, wave_base,
                           (unsigned long long*)total, heavy, out_r, out_s, capacity);
    }
    rec.after();
}

}  // namespace hj
