// Device-wide exclusive prefix scans (reduce-then-scan, three launches).
//
// Used for the partition histograms (uint32, modulo 2^32: consumers only take
// differences inside one segment, which are exact) and for match counts
// (uint64).  Replaces the paper's dynamic allocation of partition buckets and
// output (Section 3.3, "Memory allocator") with counted, contiguous placement.
#include "hj_device.h"
#include "hj_internal.h"

namespace hj {

namespace {

constexpr uint32_t kScanBlock = 256;
constexpr uint32_t kScanItems = 16;
constexpr uint32_t kScanChunk = kScanBlock * kScanItems;

template <typename T>
__global__ void __launch_bounds__(kScanBlock) k_scan_reduce(const T* __restrict__ in, uint64_t n,
                                                          T* __restrict__ partials) {
    const uint64_t base = (uint64_t)blockIdx.x * kScanChunk;
    T s = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanItems; ++k) {
        const uint64_t i = base + (uint64_t)k * kScanBlock + threadIdx.x;
        if (i < n) s += in[i];
    }
    s = wave_sum(s);
    __shared__ T wt[kScanBlock / kWave];
    if (lane_id() == 0) wt[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = 0;
        for (uint32_t w = 0; w < kScanBlock / kWave; ++w) t += wt[w];
        partials[blockIdx.x] = t;
    }
}

// One block scans the partials in place (exclusive) and writes the grand total.
template <typename T>
__global__ void __launch_bounds__(kScanBlock) k_scan_partials(T* __restrict__ partials, uint32_t nb,
                                                            T* __restrict__ total) {
    __shared__ T wt[kScanBlock / kWave];
    T carry = 0;
    for (uint32_t base = 0; base < nb; base += kScanBlock) {
        const uint32_t i = base + threadIdx.x;
        T v = i < nb ? partials[i] : T(0);
        T tot;
        T ex = block_excl_scan(v, wt, &tot);
        if (i < nb) partials[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

// Each block scans its chunk (items held per thread in consecutive order) and
// adds its partial prefix.  `in` and `out` may alias.
template <typename T>
__global__ void __launch_bounds__(kScanBlock) k_scan_apply(const T* in, T* out, uint64_t n,
                                                         const T* __restrict__ partials) {
    __shared__ T wt[kScanBlock / kWave];
    const uint64_t base = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanItems;
    T v[kScanItems];
    T s = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanItems; ++k) {
        const uint64_t i = base + k;
        v[k] = i < n ? in[i] : T(0);
        s += v[k];
    }
    T tot;
    T run = block_excl_scan(s, wt, &tot) + partials[blockIdx.x];
#pragma unroll
    for (uint32_t k = 0; k < kScanItems; ++k) {
        const uint64_t i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

template <typename T>
void scan_impl(const T* in, T* out, uint64_t n, T* partials, T* total, Recorder& rec,
               const char* name) {
    const uint64_t nb = (n + kScanChunk - 1) / kScanChunk;
    if (nb == 0) {
        rec.before(name);
        hipLaunchKernelGGL(k_scan_partials<T>, dim3(1), dim3(kScanBlock), 0, rec.stream, partials,
                           0u, total);
        rec.after();
        return;
    }
    rec.before(name);
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((uint32_t)nb), dim3(kScanBlock), 0, rec.stream, in,
                       n, partials);
    rec.after();
    rec.before(name);
    hipLaunchKernelGGL(k_scan_partials<T>, dim3(1), dim3(kScanBlock), 0, rec.stream, partials,
                       (uint32_t)nb, total);
    rec.after();
    rec.before(name);
    hipLaunchKernelGGL(k_scan_apply<T>, dim3((uint32_t)nb), dim3(kScanBlock), 0, rec.stream, in,
                       out, n, partials);
    rec.after();
}

}  // namespace

size_t scan_partials(uint64_t n) { return (size_t)((n + kScanChunk - 1) / kScanChunk) + 1; }

void scan_u32(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* partials, uint32_t* total,
              Recorder& rec) {
    scan_impl<uint32_t>(in, out, n, partials, total, rec, "scan_u32");
}

void scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* partials, uint64_t* total,
              Recorder& rec) {
    scan_impl<uint64_t>(in, out, n, partials, total, rec, "scan_u64");
}

}  // namespace hj
