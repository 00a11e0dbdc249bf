// Join server: continuous batching of join requests arriving over time.
//
// Requests (device-resident R and S, an output buffer, a device count) are
// submitted from any thread; each carries a footprint in bytes (its inputs,
// output reservation and workspace).  A dispatcher thread owns `slots`
// streams.  Whenever a slot is idle and requests are waiting, it admits
// requests from the head of the FIFO while the sum of footprints of all
// requests on the device stays within the memory cap, the batch stays within
// max_batch_jobs and its workspace fits the slot's share of the pool; the
// admitted requests run as one batch on that slot's stream (requests whose R
// fits the LDS budget in one multi-job direct kernel, the others one after
// another with their own parameters).  Batches on different slots overlap on
// the device; a finished batch (polled through its event) releases its
// footprint and records each request's completion time, so requests that
// arrive while others are on the GPU are admitted as soon as a slot and memory
// free up.  A request whose footprint alone exceeds the cap, or whose
// workspace exceeds a slot, is rejected.  The admission policy itself lives in
// server_core.h (no device state), which a host test drives with a virtual
// clock; this file runs its batches on HIP streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/hj.h"
#include "engine.h"
#include "hj_internal.h"
#include "server_core.h"

using namespace hj::eng;

namespace {

using Clock = std::chrono::steady_clock;

// What the device needs of a request (the core keeps its ticket, footprint,
// workspace need and arrival).
struct Request {
    hj_job job;
    bool probe = false;  // a probe of `table` by job.S (else a join of job.R and job.S)
    hj_table table{};
    Plan plan;
};

// Device resources of a slot (its admission state is the core's).
struct SlotDev {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    hj::DirectJob* h_djobs = nullptr;  // pinned, max_batch entries
    uint32_t* h_items = nullptr;       // pinned, max_items entries
    uint64_t* h_err = nullptr;         // pinned: the batch's device error word, copied back at its end
    char* ws = nullptr;                // this slot's workspace share: [error word][jobs][items][pipeline]
};

using Core = hj::srv::Core<Request>;

// Direct work items a slot can hold (a direct job with |S| beyond the per-job
// share of this runs through the pipeline path instead).
constexpr uint32_t kItemsPerJob = 64;

}  // namespace

struct hj_server {
    hj_server_config cfg{};
    std::vector<SlotDev> slots;
    size_t slot_ws = 0, slot_djobs_off = 0, slot_items_off = 0, slot_pipe_off = 0;
    std::mutex mu;
    std::condition_variable cv;
    Core* core = nullptr;  // guarded by mu
    Clock::time_point t0;
    bool stop = false;
    hj_status fatal = HJ_OK;
    std::thread worker;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

// Enqueues a slot's admitted requests (reqs) on its stream.
hj_status launch_slot(hj_server* sv, SlotDev& s, const std::vector<Core::Req>& reqs) {
    uint32_t nd = 0, items = 0;
    std::vector<size_t> piped;
    for (size_t i = 0; i < reqs.size(); ++i) {
        const Request& r = reqs[i].payload;
        const uint32_t it = (r.job.R.n && r.job.S.n) ? (uint32_t)cdiv(r.job.S.n, hj::kJoinChunk) : 0u;
        if (!r.probe && r.plan.phj && r.plan.passes == 0 && items + it <= sv->cfg.max_batch_jobs * kItemsPerJob) {
            hj::DirectJob& d = s.h_djobs[nd];
            std::memset(&d, 0, sizeof d);
            d.rk = r.job.R.key;
            d.rr = r.job.R.rid;
            d.sk = r.job.S.key;
            d.sr = r.job.S.rid;
            d.out_r = r.job.out.rid_r;
            d.out_s = r.job.out.rid_s;
            d.capacity = r.job.out.capacity;
            d.count = r.job.d_count;
            d.n_r = (uint32_t)r.job.R.n;
            d.n_s = (uint32_t)r.job.S.n;
            d.item0 = items;
            for (uint32_t k = 0; k < it; ++k) s.h_items[items + k] = nd;
            items += it;
            ++nd;
        } else {
            piped.push_back(i);
        }
    }
    hj::Recorder rec;
    uint64_t* d_err = (uint64_t*)s.ws;
    init_recorder(rec, s.stream, d_err, false);
    hj::zero_pair(d_err, nullptr, rec);  // one error word for the slot's batch
    hj::DirectJob* d_djobs = (hj::DirectJob*)(s.ws + sv->slot_djobs_off);
    uint32_t* d_items = (uint32_t*)(s.ws + sv->slot_items_off);
    if (nd) {
        hipError_t e = hipMemcpyAsync(d_djobs, s.h_djobs, sizeof(hj::DirectJob) * nd, hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess && items)
            e = hipMemcpyAsync(d_items, s.h_items, sizeof(uint32_t) * items, hipMemcpyHostToDevice, s.stream);
        if (e != hipSuccess) return fail(HJ_ERR_DEVICE, "server upload failed: %s", hipGetErrorString(e));
        uint32_t cap = 256;
        for (const Core::Req& q : reqs)
            if (q.payload.plan.phj && q.payload.plan.passes == 0) cap = std::max(cap, q.payload.plan.lds_cap);
        hj::direct_zero(d_djobs, nd, rec);
        hj::direct_join(d_djobs, d_items, items, cap, rec);
    }
    for (size_t i : piped) {
        const Request& r = reqs[i].payload;
        if (r.probe)
            run_probe(r.plan, r.table, r.job.S, r.job.out, s.ws + sv->slot_pipe_off, r.job.d_count, rec);
        else
            run_join(r.plan, r.job.R, r.job.S, r.job.out, s.ws + sv->slot_pipe_off, r.job.d_count, rec);
    }
    if (rec.err != hipSuccess) return fail(HJ_ERR_DEVICE, "server launch failed: %s", hipGetErrorString(rec.err));
    *s.h_err = 0;
    hipError_t e = hipMemcpyAsync(s.h_err, d_err, sizeof(uint64_t), hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
    if (e != hipSuccess) return fail(HJ_ERR_DEVICE, "server event failed: %s", hipGetErrorString(e));
    return HJ_OK;
}

void dispatcher(hj_server* sv) {
    std::unique_lock<std::mutex> lk(sv->mu);
    Core& c = *sv->core;
    while (true) {
        // retire finished batches
        bool any_busy = false;
        for (uint32_t i = 0; i < sv->slots.size(); ++i) {
            if (!c.slots[i].busy) continue;
            SlotDev& s = sv->slots[i];
            hipError_t q = hipEventQuery(s.done);
            if (q == hipErrorNotReady) {
                any_busy = true;
                continue;
            }
            // a set error word fails this batch's requests; the server goes on
            const bool ok = q == hipSuccess && sv->fatal == HJ_OK && *s.h_err == 0;
            c.retire(i, ok, sv->now(), HJ_ERR_DEVICE);
            if (q != hipSuccess && sv->fatal == HJ_OK) sv->fatal = HJ_ERR_DEVICE;
            sv->cv.notify_all();
        }
        // admit waiting requests into idle slots
        bool rejected_any = false;
        const std::vector<uint32_t> to_launch = c.admit(sv->now(), &rejected_any);
        if (!to_launch.empty()) any_busy = true;
        // a rejection can leave nothing pending or in flight: wake drain()
        if (rejected_any) sv->cv.notify_all();
        if (!to_launch.empty()) {
            // A busy slot's requests change only when this thread retires it,
            // so they can be read without the lock; submitters need not wait
            // for the launches.
            lk.unlock();
            hj_status st = HJ_OK;
            for (uint32_t i : to_launch) {
                const hj_status e = launch_slot(sv, sv->slots[i], c.slots[i].reqs);
                if (st == HJ_OK) st = e;
            }
            lk.lock();
            if (st != HJ_OK && sv->fatal == HJ_OK) {
                sv->fatal = st;
                sv->cv.notify_all();
            }
        }
        if (sv->stop && c.pending.empty() && !any_busy) break;
        if (any_busy) {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            sv->cv.wait_for(lk, std::chrono::microseconds(200),
                            [&] { return sv->stop || !c.pending.empty(); });
        }
    }
}

void destroy(hj_server* sv) {
    for (SlotDev& s : sv->slots) {
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        if (s.h_djobs) (void)hipHostFree(s.h_djobs);
        if (s.h_items) (void)hipHostFree(s.h_items);
        if (s.h_err) (void)hipHostFree(s.h_err);
    }
    delete sv->core;
    delete sv;
}

}  // namespace

extern "C" {

hj_status hj_server_create(const hj_server_config* cfg, void* ws, size_t ws_bytes, hj_server** out) {
    if (!out) return fail(HJ_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(HJ_ERR_INVALID, "config is NULL");
    if (cfg->slots == 0 || cfg->slots > 16) return fail(HJ_ERR_INVALID, "slots must be in 1..16");
    if (cfg->max_batch_jobs == 0) return fail(HJ_ERR_INVALID, "max_batch_jobs must be > 0");
    if (cfg->flags != 0) return fail(HJ_ERR_INVALID, "flags must be 0");
    if (!ws || (uintptr_t)ws % kAlign) return fail(HJ_ERR_INVALID, "workspace must be non-NULL and 256-byte aligned");
    hj_server* sv = new (std::nothrow) hj_server;
    if (!sv) return fail(HJ_ERR_DEVICE, "out of host memory");
    sv->cfg = *cfg;
    sv->slots.resize(cfg->slots);
    sv->slot_djobs_off = align_up(sizeof(uint64_t));
    sv->slot_items_off = sv->slot_djobs_off + align_up(sizeof(hj::DirectJob) * cfg->max_batch_jobs);
    sv->slot_pipe_off = sv->slot_items_off + align_up(sizeof(uint32_t) * cfg->max_batch_jobs * kItemsPerJob);
    sv->slot_ws = (ws_bytes / cfg->slots) / kAlign * kAlign;
    if (sv->slot_ws <= sv->slot_pipe_off) {
        destroy(sv);
        return fail(HJ_ERR_WORKSPACE, "workspace too small for %u slots", cfg->slots);
    }
    sv->core = new (std::nothrow)
        Core(hj::srv::CoreConfig{cfg->slots, cfg->max_batch_jobs, cfg->mem_cap_bytes, sv->slot_ws - sv->slot_pipe_off});
    if (!sv->core) {
        destroy(sv);
        return fail(HJ_ERR_DEVICE, "out of host memory");
    }
    sv->t0 = Clock::now();
    for (uint32_t i = 0; i < cfg->slots; ++i) {
        SlotDev& s = sv->slots[i];
        s.ws = (char*)ws + i * sv->slot_ws;
        hipError_t e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_djobs, sizeof(hj::DirectJob) * cfg->max_batch_jobs,
                                               hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc((void**)&s.h_items, sizeof(uint32_t) * cfg->max_batch_jobs * kItemsPerJob,
                              hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_err, sizeof(uint64_t), hipHostMallocDefault);
        if (e != hipSuccess) {
            destroy(sv);
            return fail(HJ_ERR_DEVICE, "server setup failed: %s", hipGetErrorString(e));
        }
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    sv->worker = std::thread([sv, dev] {
        (void)hipSetDevice(dev);
        dispatcher(sv);
    });
    *out = sv;
    clear_error();
    return HJ_OK;
}

hj_status hj_server_submit(hj_server* sv, const hj_job* job, const hj_params* params, uint64_t footprint,
                           uint64_t* ticket) {
    if (!sv || !job || !params || !ticket) return fail(HJ_ERR_INVALID, "server, job, params and ticket must be given");
    if (job->R.n > kMaxRows || job->S.n > kMaxRows) return fail(HJ_ERR_INVALID, "relations must have < 2^31 tuples");
    if ((job->R.n && (!job->R.key || !job->R.rid)) || (job->S.n && (!job->S.key || !job->S.rid)))
        return fail(HJ_ERR_INVALID, "relation with tuples but a NULL array");
    if (job->out.capacity && (!job->out.rid_r || !job->out.rid_s))
        return fail(HJ_ERR_INVALID, "out has capacity but a NULL array");
    if (!job->d_count) return fail(HJ_ERR_INVALID, "d_count is NULL");
    Request r;
    hj_status st = check_params(params, job->R.n, job->S.n, &r.plan);
    if (st != HJ_OK) return st;
    r.job = *job;
    const size_t ws = ws_bytes_for(r.plan, job->R.n, job->S.n);
    // the bytes the request holds on the device are at least its own arrays and workspace
    footprint = std::max(footprint, hj::srv::least_footprint(job->R.n, job->S.n, job->out.capacity, ws));
    {
        std::lock_guard<std::mutex> g(sv->mu);
        if (sv->fatal != HJ_OK) return fail(sv->fatal, "server stopped after a device error");
        *ticket = sv->core->submit(footprint, ws, sv->now(), r);
    }
    sv->cv.notify_all();
    clear_error();
    return HJ_OK;
}

hj_status hj_server_submit_probe(hj_server* sv, const hj_table* table, const hj_rel* S, const hj_out* out,
                                 uint64_t* d_count, uint64_t footprint, uint64_t* ticket) {
    if (!sv || !table || !S || !out || !d_count || !ticket)
        return fail(HJ_ERR_INVALID, "server, table, S, out, d_count and ticket must be given");
    if (S->n > kMaxRows) return fail(HJ_ERR_INVALID, "relations must have < 2^31 tuples");
    if (S->n && (!S->key || !S->rid)) return fail(HJ_ERR_INVALID, "S has tuples but a NULL array");
    if (out->capacity && (!out->rid_r || !out->rid_s))
        return fail(HJ_ERR_INVALID, "out has capacity but a NULL array");
    Request r;
    hj_status st = table_plan(table, S->n, &r.plan);
    if (st != HJ_OK) return st;
    r.probe = true;
    r.table = *table;
    r.job.R = hj_rel{table->r_key, table->r_rid, table->n_r};
    r.job.S = *S;
    r.job.out = *out;
    r.job.d_count = d_count;
    const size_t ws = probe_bytes_for(r.plan, table->n_r, S->n);
    // the table stays resident and is the caller's; S, the output and the workspace are the request's
    footprint = std::max(footprint, hj::srv::least_footprint(0, S->n, out->capacity, ws));
    {
        std::lock_guard<std::mutex> g(sv->mu);
        if (sv->fatal != HJ_OK) return fail(sv->fatal, "server stopped after a device error");
        *ticket = sv->core->submit(footprint, ws, sv->now(), r);
    }
    sv->cv.notify_all();
    clear_error();
    return HJ_OK;
}

hj_status hj_server_poll(hj_server* sv, uint64_t* tickets, int32_t* status, double* latency_s, double* queue_s,
                         uint32_t max, uint32_t* n) {
    if (!sv || !n || (max && (!tickets || !status || !latency_s || !queue_s)))
        return fail(HJ_ERR_INVALID, "bad poll arguments");
    std::lock_guard<std::mutex> g(sv->mu);
    std::vector<hj::srv::Finished>& done = sv->core->done;
    const uint32_t k = (uint32_t)std::min<size_t>(max, done.size());
    for (uint32_t i = 0; i < k; ++i) {
        tickets[i] = done[i].ticket;
        status[i] = done[i].status;
        latency_s[i] = done[i].latency_s;
        queue_s[i] = done[i].queue_s;
    }
    done.erase(done.begin(), done.begin() + k);
    *n = k;
    return sv->fatal;
}

hj_status hj_server_drain(hj_server* sv) {
    if (!sv) return fail(HJ_ERR_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv.wait(lk, [&] { return sv->core->idle() || sv->fatal != HJ_OK; });
    return sv->fatal;
}

hj_status hj_server_stats(hj_server* sv, uint64_t* completed, uint64_t* rejected, uint64_t* batches,
                          uint64_t* bytes_in_use) {
    if (!sv) return fail(HJ_ERR_INVALID, "server is NULL");
    std::lock_guard<std::mutex> g(sv->mu);
    if (completed) *completed = sv->core->completed;
    if (rejected) *rejected = sv->core->rejected;
    if (batches) *batches = sv->core->batches;
    if (bytes_in_use) *bytes_in_use = sv->core->used;
    return HJ_OK;
}

void hj_server_destroy(hj_server* sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->stop = true;
    }
    sv->cv.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    for (SlotDev& s : sv->slots)
        if (s.stream) (void)hipStreamSynchronize(s.stream);
    destroy(sv);
}

}  // extern "C"
