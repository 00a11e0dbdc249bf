// C ABI of the single join (include/hj.h): thin wrappers over the engine.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hj.h"
#include "engine.h"
#include "hj_internal.h"

using namespace hj::eng;


namespace hj {

void Recorder::before(const char* name) {
    cur = name;
    if (timed && n < cap) {
        names[n] = name;
        hipError_t e = hipEventRecord(ev[2 * n], stream);
        if (e != hipSuccess && err == hipSuccess) err = e;
    }
}

void Recorder::after() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess && err == hipSuccess) err = e;
    if (fail_phase && cur && std::strcmp(fail_phase, cur) == 0 && err == hipSuccess) err = hipErrorLaunchFailure;
    if (timed && n < cap) {
        e = hipEventRecord(ev[2 * n + 1], stream);
        if (e != hipSuccess && err == hipSuccess) err = e;
    }
    ++n;
}

}  // namespace hj

namespace {
hj_status ws_error(uint64_t werr) {
    return fail(HJ_ERR_DEVICE, "device error word 0x%llx: %s", (unsigned long long)werr,
                (werr & hj::kErrLookback) ? "a chained scan gave up waiting for a predecessor's status; "
                                            "the output of the call is not valid"
                                          : "unknown device-side failure");
}
}  // namespace

extern "C" {

void hj_default_params(hj_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->algo = HJ_PHJ;
    p->passes = 2;
    p->bits[0] = 6;
    p->bits[1] = 6;
    p->hash = HJ_HASH_IDENTITY;
    p->tile = 0;
    p->lds_cap = 0;
    p->flags = 0;
}

size_t hj_workspace_bytes(const hj_params* p, uint64_t n_r, uint64_t n_s) {
    Plan pl;
    if (check_params(p, n_r, n_s, &pl) != HJ_OK) return 0;
    if (n_r > kMaxRows || n_s > kMaxRows) {
        fail(HJ_ERR_INVALID, "relations must have fewer than 2^31 tuples");
        return 0;
    }
    return ws_bytes_for(pl, n_r, n_s);
}

hj_status hj_resolve_params(const hj_params* p, uint64_t n_r, uint64_t n_s, hj_params* out) {
    if (!out) return fail(HJ_ERR_INVALID, "out is NULL");
    Plan pl;
    const hj_status st = check_params(p, n_r, n_s, &pl);
    if (st != HJ_OK) return st;
    if (n_r > kMaxRows || n_s > kMaxRows) return fail(HJ_ERR_INVALID, "relations must have fewer than 2^31 tuples");
    *out = pl.res;
    clear_error();
    return HJ_OK;
}

size_t hj_table_bytes(const hj_params* p, uint64_t n_r) {
    Plan pl;
    if (check_params(p, n_r, n_r, &pl) != HJ_OK) return 0;
    if (n_r > kMaxRows) {
        fail(HJ_ERR_INVALID, "relations must have fewer than 2^31 tuples");
        return 0;
    }
    return table_bytes_for(pl, n_r);
}

hj_status hj_build(const hj_params* p, const hj_rel* R, void* ws, size_t ws_bytes, void* stream,
                   hj_table* table) {
    if (!R || !table) return fail(HJ_ERR_INVALID, "R and table must not be NULL");
    Plan pl;
    hj_status st = check_params(p, R->n, R->n, &pl);
    if (st != HJ_OK) return st;
    if (R->n > kMaxRows) return fail(HJ_ERR_INVALID, "relations must have fewer than 2^31 tuples");
    if (R->n && (!R->key || !R->rid)) return fail(HJ_ERR_INVALID, "R has tuples but a NULL array");
    const size_t need = table_bytes_for(pl, R->n);
    if (!ws || ws_bytes < need)
        return fail(HJ_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : 0);
    if ((uintptr_t)ws % kAlign) return fail(HJ_ERR_INVALID, "workspace must be 256-byte aligned");
    hj::Recorder rec;
    init_recorder(rec, (hipStream_t)stream, (uint64_t*)ws, true);
    (void)hipGetLastError();
    run_build(pl, *R, ws, rec);
    if (rec.err != hipSuccess) return fail(HJ_ERR_DEVICE, "launch failed: %s", hipGetErrorString(rec.err));
    hj_table t{};
    t.params = pl.res;
    t.n_r = R->n;
    t.r_key = R->key;
    t.r_rid = R->rid;
    t.ws = ws;
    t.ws_bytes = ws_bytes;
    *table = t;
    clear_error();
    return HJ_OK;
}


size_t hj_probe_workspace_bytes(const hj_table* table, uint64_t n_s) {
    Plan pl;
    if (table_plan(table, n_s, &pl) != HJ_OK) return 0;
    if (n_s > kMaxRows) {
        fail(HJ_ERR_INVALID, "relations must have fewer than 2^31 tuples");
        return 0;
    }
    return probe_bytes_for(pl, table->n_r, n_s);
}

hj_status hj_probe(const hj_table* table, const hj_rel* S, const hj_out* out, void* ws, size_t ws_bytes,
                   uint64_t* d_count, void* stream) {
    if (!S || !out) return fail(HJ_ERR_INVALID, "S and out must not be NULL");
    Plan pl;
    hj_status st = table_plan(table, S->n, &pl);
    if (st != HJ_OK) return st;
    if (S->n > kMaxRows) return fail(HJ_ERR_INVALID, "relations must have fewer than 2^31 tuples");
    if (S->n && (!S->key || !S->rid)) return fail(HJ_ERR_INVALID, "S has tuples but a NULL array");
    if (out->capacity && (!out->rid_r || !out->rid_s))
        return fail(HJ_ERR_INVALID, "out has capacity but a NULL array");
    if (!d_count) return fail(HJ_ERR_INVALID, "d_count is NULL");
    const size_t need = probe_bytes_for(pl, table->n_r, S->n);
    if (!ws || ws_bytes < need)
        return fail(HJ_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : 0);
    if ((uintptr_t)ws % kAlign) return fail(HJ_ERR_INVALID, "workspace must be 256-byte aligned");
    hj::Recorder rec;
    init_recorder(rec, (hipStream_t)stream, (uint64_t*)ws, true);
    (void)hipGetLastError();
    run_probe(pl, *table, *S, *out, ws, d_count, rec);
    if (rec.err != hipSuccess) return fail(HJ_ERR_DEVICE, "launch failed: %s", hipGetErrorString(rec.err));
    clear_error();
    return HJ_OK;
}

hj_status hj_join(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out, void* ws,
                  size_t ws_bytes, uint64_t* d_count, void* stream) {
    hj::Recorder rec;
    init_recorder(rec, (hipStream_t)stream, (uint64_t*)ws, true);
    return launch_join(p, R, S, out, ws, ws_bytes, d_count, rec);
}

hj_status hj_join_sync(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out, void* ws,
                       size_t ws_bytes, uint64_t* d_count, uint64_t* h_count, void* stream) {
    if (!h_count) return fail(HJ_ERR_INVALID, "h_count is NULL");
    hj_status st = hj_join(p, R, S, out, ws, ws_bytes, d_count, stream);
    if (st != HJ_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    uint64_t werr = 0;
    hipError_t e = hipMemcpyAsync(h_count, d_count, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&werr, ws, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(HJ_ERR_DEVICE, "synchronisation failed: %s", hipGetErrorString(e));
    if (werr) return ws_error(werr);
    if (*h_count > out->capacity)
        return fail(HJ_ERR_CAPACITY, "%llu pairs do not fit capacity %llu",
                    (unsigned long long)*h_count, (unsigned long long)out->capacity);
    return HJ_OK;
}

hj_status hj_join_timed(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out, void* ws,
                        size_t ws_bytes, uint64_t* d_count, void* stream, const char** names, float* ms,
                        uint32_t max_launches, uint32_t* n_launches) {
    if (!names || !ms || !n_launches || max_launches == 0)
        return fail(HJ_ERR_INVALID, "timing arrays must be given");
    std::vector<hipEvent_t> ev(2ull * max_launches, nullptr);
    for (auto& e : ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto& x : ev)
                if (x) (void)hipEventDestroy(x);
            return fail(HJ_ERR_DEVICE, "hipEventCreate failed");
        }
    }
    hj::Recorder rec;
    init_recorder(rec, (hipStream_t)stream, (uint64_t*)ws, true);
    rec.timed = true;
    rec.cap = max_launches;
    rec.names = names;
    rec.ev = ev.data();
    hj_status st = launch_join(p, R, S, out, ws, ws_bytes, d_count, rec);
    if (st == HJ_OK) {
        hipError_t e = hipStreamSynchronize(rec.stream);
        if (e != hipSuccess) st = fail(HJ_ERR_DEVICE, "synchronisation failed: %s", hipGetErrorString(e));
    }
    const uint32_t n = std::min(rec.n, max_launches);
    *n_launches = rec.n;
    for (uint32_t i = 0; st == HJ_OK && i < n; ++i) {
        float t = 0;
        (void)hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]);
        ms[i] = t;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    return st;
}

hj_status hj_model_seconds(const hj_params* p, uint64_t n_r, uint64_t n_s, uint64_t pairs, double* seconds) {
    if (!seconds) return fail(HJ_ERR_INVALID, "seconds is NULL");
    Plan pl;
    const hj_status st = check_params(p, n_r, n_s, &pl);
    if (st != HJ_OK) return st;
    if (n_r > kMaxRows || n_s > kMaxRows) return fail(HJ_ERR_INVALID, "relations must have fewer than 2^31 tuples");
    *seconds = model_seconds(pl, n_r, n_s, (double)pairs);
    clear_error();
    return HJ_OK;
}

hj_status hj_workspace_status(const void* ws, void* stream) {
    if (!ws || (uintptr_t)ws % kAlign) return fail(HJ_ERR_INVALID, "workspace must be non-NULL and 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    uint64_t werr = 0;
    hipError_t e = hipMemcpyAsync(&werr, ws, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(HJ_ERR_DEVICE, "synchronisation failed: %s", hipGetErrorString(e));
    if (werr) return ws_error(werr);
    clear_error();
    return HJ_OK;
}

const char* hj_status_str(hj_status s) {
    switch (s) {
        case HJ_OK: return "ok";
        case HJ_ERR_INVALID: return "invalid argument";
        case HJ_ERR_CAPACITY: return "output capacity exceeded";
        case HJ_ERR_WORKSPACE: return "workspace too small";
        case HJ_ERR_DEVICE: return "device error";
        case HJ_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* hj_last_error(void) { return hj::eng::last_error(); }

uint32_t hj_version(void) { return 100; }

}  // extern "C"
