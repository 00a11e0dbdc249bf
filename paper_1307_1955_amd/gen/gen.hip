// Device side of the seeded input generators (see gen/__init__.py for the
// definitions).  Holds only input generation -- no hashing for the join, no
// partitioning, no joining -- and computes, element for element, the same
// values as the numpy side:
//   draw(key, i)      = mix64(key + (i + 1) * GAMMA)      (SplitMix64 output i)
//   uniform in [lo, lo + m): lo + ((draw >> 32) * m >> 32)
//   permutation of [0, n): 4-round Feistel network on 2h bits + cycle walking
//   Zipf rank: 1 + first index whose CDF entry exceeds (draw >> 11) * 2^-53
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * kGamma); }

struct Feistel {
    uint64_t rk[4];
    uint32_t h;
    __device__ __forceinline__ uint64_t enc(uint64_t v) const {
        const uint64_t mask = (1ull << h) - 1;
        uint64_t l = v >> h, r = v & mask;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint64_t f = mix64(rk[i] ^ r) & mask;
            const uint64_t nl = r;
            r = l ^ f;
            l = nl;
        }
        return (l << h) | r;
    }
};

__global__ void k_perm_keys(int32_t* __restrict__ out, uint64_t n, Feistel f, int64_t offset) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t y = f.enc(i);
        while (y >= n) y = f.enc(y);  // cycle walking: terminates, the network is a bijection
        out[i] = (int32_t)((int64_t)y + offset);
    }
}

__global__ void k_uniform(int32_t* __restrict__ out, uint64_t count, uint64_t key, int64_t lo, uint64_t m) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint64_t d = draw(key, i) >> 32;
        out[i] = (int32_t)(lo + (int64_t)((d * m) >> 32));
    }
}

__global__ void k_zipf(int32_t* __restrict__ out, uint64_t count, uint64_t key,
                       const double* __restrict__ cdf, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const double u = (double)(draw(key, i) >> 11) * (1.0 / 9007199254740992.0);
        uint64_t lo = 0, hi = n;  // first index with cdf > u, in [0, n]
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (cdf[mid] > u) hi = mid; else lo = mid + 1;
        }
        if (lo > n - 1) lo = n - 1;
        out[i] = (int32_t)(lo + 1);
    }
}

__global__ void k_iota(int32_t* __restrict__ out, uint64_t n, int64_t start) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = (int32_t)(start + (int64_t)i);
}

uint32_t grid_for(uint64_t n) {
    uint64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    return b ? (uint32_t)b : 1u;
}

int finish() { return hipGetLastError() == hipSuccess ? 0 : 1; }

}  // namespace

extern "C" {

// out[i] = perm(i) + offset for i < n; rk: the 4 round keys, h: half width in bits.
int hjgen_perm_keys(int32_t* out, uint64_t n, const uint64_t* rk, uint32_t h, int64_t offset, void* stream) {
    if (n == 0) return 0;
    if (!out || !rk || h == 0 || h > 31) return 2;
    Feistel f;
    for (int i = 0; i < 4; ++i) f.rk[i] = rk[i];
    f.h = h;
    hipLaunchKernelGGL(k_perm_keys, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, out, n, f, offset);
    return finish();
}

int hjgen_uniform(int32_t* out, uint64_t count, uint64_t key, int64_t lo, uint64_t m, void* stream) {
    if (count == 0) return 0;
    if (!out || m == 0 || m > (1ull << 32)) return 2;
    hipLaunchKernelGGL(k_uniform, dim3(grid_for(count)), dim3(256), 0, (hipStream_t)stream, out, count, key, lo, m);
    return finish();
}

int hjgen_zipf(int32_t* out, uint64_t count, uint64_t key, const double* cdf, uint64_t n, void* stream) {
    if (count == 0) return 0;
    if (!out || !cdf || n == 0) return 2;
    hipLaunchKernelGGL(k_zipf, dim3(grid_for(count)), dim3(256), 0, (hipStream_t)stream, out, count, key, cdf, n);
    return finish();
}

int hjgen_iota(int32_t* out, uint64_t n, int64_t start, void* stream) {
    if (n == 0) return 0;
    if (!out) return 2;
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, out, n, start);
    return finish();
}

}  // extern "C"
