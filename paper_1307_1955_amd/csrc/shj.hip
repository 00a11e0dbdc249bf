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

struct PowStep {
    uint64_t mask;
    __device__ __forceinline__ uint64_t operator()(uint64_t s) const { return (s + 1) & mask; }
};

__device__ __forceinline__ uint64_t home_slot(int32_t k, uint32_t log2_slots) {
    return (uint64_t)(slot_hash(k) >> (32 - log2_slots));
}

__global__ void __launch_bounds__(256) k_shj_build(const int32_t* __restrict__ key, uint64_t n,
                                                  uint64_t* __restrict__ table, uint32_t* __restrict__ next,
                                                  uint32_t log2_slots, HotKeys* hot) {
    constexpr uint32_t kWaves = 256 / kWave;
    __shared__ WavePush::Run runs[kWaves];
    const PowStep step{(1ull << log2_slots) - 1};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    WavePush push;
    push.hot_keys = hot;
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

// An S tuple whose chain is longer than lim is registered in hs as heavy.  When
// the build recorded its key as hot (hk[0..nhk), LDS) with more than lim rows
// (hr: the recorded lower bound of the chain length), it is registered without
// walking the chain; otherwise the walk decides.
// hs->n must be zero and visible to the block before the call.
template <bool kRids>
__device__ __forceinline__ void shj_probe(const int32_t* __restrict__ s_key, const int32_t* __restrict__ s_rid,
                                          uint64_t begin, uint64_t n_s, const uint64_t* __restrict__ table,
                                          const uint32_t* __restrict__ next, uint32_t log2_slots, uint32_t lim,
                                          const int32_t* hk, const uint32_t* hr, uint32_t nhk, HeavySet* hs,
                                          int32_t* q, int32_t* qr,
                                          uint32_t* head, uint32_t* cnt) {
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
            if (head[u] != kNotFound) {
                uint32_t hot_rows = 0;
                if (!(head[u] & kLast))  // a chain of one row is never heavy
                    for (uint32_t i = 0; i < nhk; ++i) hot_rows = hk[i] == q[u] ? max(hot_rows, hr[i]) : hot_rows;
                cnt[u] = hot_rows > lim ? register_heavy(next, head[u], q[u], kRids ? qr[u] : 0, hs)
                                        : heavy_or_len(next, head[u], lim, q[u], kRids ? qr[u] : 0, hs);
            }
        }
    }
}

// The build's hot keys into LDS (before the barrier that publishes hs->n = 0).
__device__ __forceinline__ void load_hot(const HotKeys* hot, int32_t* hk, uint32_t* hr, uint32_t* nhk) {
    const uint32_t n = min(hot->n, kHotKeys);
    if (threadIdx.x == 0) *nhk = n;
    if (threadIdx.x < n) {
        hk[threadIdx.x] = hot->key[threadIdx.x];
        hr[threadIdx.x] = hot->rows[threadIdx.x];
    }
}

__device__ __forceinline__ uint32_t count_of(uint32_t c, const HeavySet* hs) {
    return is_heavy(c) ? hs->cnt[c & ~kHeavyBit] : c;
}

__global__ void __launch_bounds__(kShjBlock) k_shj_count(const int32_t* __restrict__ s_key, uint64_t n_s,
                                                        const uint64_t* __restrict__ table,
                                                        const uint32_t* __restrict__ next,
                                                        uint32_t log2_slots, const int32_t* __restrict__ r_key,
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
    shj_probe<false>(s_key, nullptr, begin, n_s, table, next, log2_slots, heavy_limit(n_r), hk, hr, nhk, &hs, q, qr,
                     head, c);
    heavy_counts<kShjBlock, kHeavyV>(r_key, n_r, &hs);
    uint64_t cnt = 0;
#pragma unroll
    for (uint32_t u = 0; u < kSU; ++u) cnt += count_of(c[u], &hs);
    cnt = wave_sum(cnt);
    if (lane_id() == 0) wave_cnt[(uint64_t)blockIdx.x * kShjWavesPerBlock + w] = cnt;
}

// ---- Heavy S tuples shared by all workgroups (one-pass output) ----
// A workgroup hands the heavy tuples it registered to the queue (hand_off);
// every workgroup, once its tile is written, runs help_heavy: for each queued
// tuple it claims chunks of R and writes the tuple's matches in them, each
// scan step reserving its slots on the running total (one-pass output has no
// fixed order, so no count is needed first).  Nothing waits: a workgroup
// takes what is unclaimed and leaves; the workgroup that queued a tuple runs
// help_heavy too, so every chunk is written before the launch ends.

// Moves this block's registered heavy tuples to the queue while it has room
// (marked in hs->queued); a tuple that finds the queue full stays with the
// block's own scan of R (heavy_counts / heavy_writes).  All threads call it
// after the registrations.
__device__ __forceinline__ void hand_off(HeavyQueue* Q, HeavySet* hs) {
    __syncthreads();  // registrations done
    const uint32_t ne = min(hs->n, kMaxHeavy);
    if (threadIdx.x < ne) {
        const uint32_t idx = atomicAdd(&Q->n, 1u);
        if (idx < kHeavyJobs) {
            HeavyJob* J = &Q->job[idx];
            J->key = hs->key[threadIdx.x];
            J->srid = hs->srid[threadIdx.x];
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

template <uint32_t kBlock>
__device__ __forceinline__ void help_heavy(HeavyQueue* Q, const int32_t* __restrict__ rk,
                                           const int32_t* __restrict__ rr, uint64_t n_r,
                                           unsigned long long* __restrict__ total, uint64_t capacity,
                                           int32_t* __restrict__ out_r, int32_t* __restrict__ out_s, uint32_t* sh) {
    constexpr uint32_t kWaves = kBlock / kWave;
    constexpr uint32_t kV = kHeavyV;
    static_assert(kHeavyJobs <= kBlock, "one thread per queued tuple looks for open work");
    uint32_t* cnt = sh + 8;  // kV * kWaves per-wave hit counts of a step
    const uint32_t w = threadIdx.x / kWave;
    const uint32_t nchunks = (uint32_t)((n_r + kHelpChunk - 1) / kHelpChunk);
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
        if (threadIdx.x < nj) {
            HeavyJob* J = &Q->job[threadIdx.x];
            if (__hip_atomic_load(&J->valid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &&
                __hip_atomic_load(&J->write_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < nchunks)
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
        }
        __syncthreads();
        const int32_t k = (int32_t)sh[2], srid = (int32_t)sh[3];
        while (true) {
            const uint32_t c = claim_chunk(&J->write_next, sh);
            if (c >= nchunks) break;
            const uint64_t lo = (uint64_t)c * kHelpChunk, hi = min(lo + kHelpChunk, n_r);
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

// Write pass; kOnePass reserves the block's output with one atomic add on the
// running total instead of reading a scanned offset (see HJ_FLAG_ONE_PASS).
template <bool kOnePass>
__global__ void __launch_bounds__(kShjBlock) __attribute__((amdgpu_waves_per_eu(8))) k_shj_write(
    const int32_t* __restrict__ s_key, const int32_t* __restrict__ s_rid, uint64_t n_s,
    const uint64_t* __restrict__ table, const uint32_t* __restrict__ next, uint32_t log2_slots,
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
    shj_probe<true>(s_key, s_rid, begin, n_s, table, next, log2_slots, lim, hk, hr, nhk, &hs, q, qr, head, c);
    // with R in one chunk the queue adds no workgroups to a tuple: keep the block's own scan
    if (kOnePass && n_r > kHelpChunk) hand_off(heavy, &hs);
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
    if (kOnePass) help_heavy<kShjBlock>(heavy, r_key, r_rid, n_r, total, capacity, out_r, out_s, hs.wsum);
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

void shj_build(const int32_t* key, uint64_t n, uint64_t* table, uint32_t* next, uint32_t log2_slots,
               HotKeys* hot, Recorder& rec) {
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;  // grid-stride: a wave's pending push chain spans its rows
    if (blocks == 0) return;
    rec.before("shj_build");
    hipLaunchKernelGGL(k_shj_build, dim3((uint32_t)blocks), dim3(256), 0, rec.stream, key, n, table, next,
                       log2_slots, hot);
    rec.after();
}

void shj_count(const int32_t* s_key, uint64_t n_s, const uint64_t* table, const uint32_t* next,
               uint32_t log2_slots, const int32_t* r_key, uint64_t n_r, const HotKeys* hot, uint64_t* wave_cnt,
               Recorder& rec) {
    const uint64_t tiles = (n_s + kShjTile - 1) / kShjTile;
    if (tiles == 0) return;
    rec.before("shj_count");
    hipLaunchKernelGGL(k_shj_count, dim3((uint32_t)tiles), dim3(kShjBlock), 0, rec.stream, s_key, n_s,
                       table, next, log2_slots, r_key, n_r, hot, wave_cnt, rec.err_clear);
    rec.after();
}

void shj_write(const int32_t* s_key, const int32_t* s_rid, uint64_t n_s, const uint64_t* table,
               const uint32_t* next, uint32_t log2_slots, const int32_t* r_key, const int32_t* r_rid,
               uint64_t n_r, const HotKeys* hot, const uint64_t* wave_base, uint64_t* total, HeavyQueue* heavy,
               int32_t* out_r, int32_t* out_s, uint64_t capacity, Recorder& rec) {
    const uint64_t tiles = (n_s + kShjTile - 1) / kShjTile;
    if (tiles == 0) return;
    if (wave_base == nullptr) {
        rec.before("shj_write_1pass");
        hipLaunchKernelGGL(k_shj_write<true>, dim3((uint32_t)tiles), dim3(kShjBlock), 0, rec.stream, s_key,
                           s_rid, n_s, table, next, log2_slots, r_key, r_rid, n_r, hot, wave_base,
                           (unsigned long long*)total, heavy, out_r, out_s, capacity);
    } else {
        rec.before("shj_write");
        hipLaunchKernelGGL(k_shj_write<false>, dim3((uint32_t)tiles), dim3(kShjBlock), 0, rec.stream, s_key,
                           s_rid, n_s, table, next, log2_slots, r_key, r_rid, n_r, hot, wave_base,
                           (unsigned long long*)total, heavy, out_r, out_s, capacity);
    }
    rec.after();
}

}  // namespace hj
