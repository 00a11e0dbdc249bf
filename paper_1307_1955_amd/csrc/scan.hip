// Device-wide exclusive prefix scans in one launch (chained scan with
// decoupled look-back).
//
// Used for the partition histograms (uint32, modulo 2^32: consumers only take
// differences inside one segment, which are exact) and for match counts
// (uint64).  Replaces the paper's dynamic allocation of partition buckets and
// output (Section 3.3, "Memory allocator") with counted, contiguous placement.
//
// Each workgroup takes the next tile from a ticket counter (so every tile's
// predecessors were started before it and finish without waiting on it),
// reduces the tile, publishes the tile sum as an "aggregate" status, then walks
// back over its predecessors' statuses (one wave, 64 at a time), adding
// aggregates until it meets an "inclusive" one, publishes its own inclusive
// prefix and writes the tile's scanned values.  A status is one 64-bit word: flag in the top two bits, value
// below, written and read with single-copy-atomic device-scope accesses.  The
// state words must be zero before the launch (the callers clear them in the
// first kernel of a join).
#include "hj_device.h"
#include "hj_internal.h"

namespace hj {

namespace {

constexpr uint32_t kScanBlock = 256;
// items per thread: 8 measured best on MI355X for the 1 MB partition
// histograms and the per-wave count arrays (16: 1 us slower per scan, 2: 5 us)
constexpr uint32_t kScanItems = 8;
constexpr uint32_t kScanChunk = kScanBlock * kScanItems;
// state[0]: tile ticket; state[1 + t]: status of tile t.
template <typename T>
__global__ void __launch_bounds__(kScanBlock) k_scan(const T* in, T* out, uint64_t n, uint64_t* state,
                                                   uint32_t ntiles, T* __restrict__ total, ScanCtl ctl) {
    __shared__ T wt[kScanBlock / kWave];
    __shared__ uint32_t s_tile;
    __shared__ T s_prefix;
    if (threadIdx.x == 0) s_tile = (uint32_t)atomicAdd((unsigned long long*)state, 1ull);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint64_t base = (uint64_t)tile * kScanChunk + (uint64_t)threadIdx.x * kScanItems;
    T v[kScanItems];
    T s = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanItems; ++k) {
        const uint64_t i = base + k;
        v[k] = i < n ? in[i] : T(0);
        s += v[k];
    }
    T tot;
    T run = block_excl_scan(s, wt, &tot);
    if (threadIdx.x < kWave) {  // wave 0: publish, then look back
        const T prefix = (T)lookback_wave(state + 1, tile, (uint64_t)tot & kStatusValue, ctl);
        if (threadIdx.x == 0) {
            s_prefix = prefix;
            if (tile == ntiles - 1 && total) *total = prefix + tot;
        }
    }
    __syncthreads();
    run += s_prefix;
#pragma unroll
    for (uint32_t k = 0; k < kScanItems; ++k) {
        const uint64_t i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

template <typename T>
__global__ void k_scan_empty(T* __restrict__ total) {
    if (threadIdx.x == 0 && total) *total = 0;
}

__global__ void __launch_bounds__(256) k_zero_words(uint64_t* __restrict__ p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

template <typename T>
void scan_impl(const T* in, T* out, uint64_t n, uint64_t* state, T* total, Recorder& rec, const char* name) {
    const uint64_t nt = (n + kScanChunk - 1) / kScanChunk;
    rec.before(name);
    if (nt == 0)
        hipLaunchKernelGGL(k_scan_empty<T>, dim3(1), dim3(64), 0, rec.stream, total);
    else
        hipLaunchKernelGGL(k_scan<T>, dim3((uint32_t)nt), dim3(kScanBlock), 0, rec.stream, in, out, n, state,
                           (uint32_t)nt, total, rec.ctl);
    rec.after();
}

__global__ void k_zero_pair(uint64_t* a, uint64_t* b) {
    if (threadIdx.x == 0) {
        if (a) *a = 0;
        if (b) *b = 0;
    }
}

}  // namespace

void zero_pair(uint64_t* a, uint64_t* b, Recorder& rec) {
    if (!a && !b) return;
    rec.before("zero_pair");
    hipLaunchKernelGGL(k_zero_pair, dim3(1), dim3(64), 0, rec.stream, a, b);
    rec.after();
}

size_t scan_state_words(uint64_t n) { return (size_t)((n + kScanChunk - 1) / kScanChunk) + 1; }

void scan_u32(const uint32_t* in, uint32_t* out, uint64_t n, uint64_t* state, uint32_t* total, Recorder& rec) {
    scan_impl<uint32_t>(in, out, n, state, total, rec, "scan_u32");
}

void scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* state, uint64_t* total, Recorder& rec) {
    scan_impl<uint64_t>(in, out, n, state, total, rec, "scan_u64");
}

void zero_words(uint64_t* p, uint64_t n, Recorder& rec) {
    if (n == 0) return;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    rec.before("zero_state");
    hipLaunchKernelGGL(k_zero_words, dim3((uint32_t)blocks), dim3(256), 0, rec.stream, p, n);
    rec.after();
}

}  // namespace hj
