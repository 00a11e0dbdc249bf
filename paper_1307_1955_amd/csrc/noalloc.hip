// hj_join for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc): the join's
// workspace is a fixed array of this library in device memory instead of a
// buffer the caller brings.  The join itself is hj_join's (same kernels, same
// launch sequence, same result).
//
// The array is file-scope and holds kScratchBytes on every GPU the library
// runs on, from the first call on that GPU until the process ends.  Every call
// on one GPU shares that GPU's array: it keeps the last call's contents (the
// join's first kernel clears whatever has to start at zero), and calls that
// overlap on one GPU -- on two streams, or from two threads -- race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/hj.h"
#include "engine.h"
#include "hj_internal.h"

using namespace hj::eng;

namespace {

constexpr size_t kScratchBytes = 64ull << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint64_t scratch[kScratchBytes / sizeof(uint64_t)];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};  // device address of `scratch` on each GPU

// The device address of this GPU's copy of the array, looked up once per
// device with that device current (the array's name is a host-side stand-in).
hj_status scratch_on_current_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(HJ_ERR_DEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(HJ_ERR_UNSUPPORTED, "device %d beyond %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(HJ_ERR_DEVICE, "hipGetSymbolAddress of the fixed workspace failed: %s", hipGetErrorString(e));
        g_ptr[dev] = ptr;
    }
    *out = g_ptr[dev];
    return HJ_OK;
}

}  // namespace

extern "C" {

hj_status hj_join_noalloc(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out,
                          uint64_t* d_count, void* stream) {
    // sizes first, on the host: nothing touches a device before they fit
    if (!R || !S) return fail(HJ_ERR_INVALID, "R and S must not be NULL");
    Plan pl;
    hj_status st = check_params(p, R->n, S->n, &pl);
    if (st != HJ_OK) return st;
    if (R->n > kMaxRows || S->n > kMaxRows) return fail(HJ_ERR_INVALID, "relations must have fewer than 2^31 tuples");
    const size_t need = ws_bytes_for(pl, R->n, S->n);
    if (need > kScratchBytes)
        return fail(HJ_ERR_WORKSPACE,
                    "hj_join_noalloc: |R| = %llu, |S| = %llu need %zu bytes of workspace, above its fixed %zu bytes "
                    "(use hj_join with a workspace of hj_workspace_bytes)",
                    (unsigned long long)R->n, (unsigned long long)S->n, need, kScratchBytes);
    void* ws = nullptr;
    st = scratch_on_current_device(&ws);
    if (st != HJ_OK) return st;
    hj::Recorder rec;
    init_recorder(rec, (hipStream_t)stream, (uint64_t*)ws, true);
    return launch_join(p, R, S, out, ws, kScratchBytes, d_count, rec);
}

}  // extern "C"
