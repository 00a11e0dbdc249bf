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
// workspace exceeds a slot, is rejected.
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

using namespace hj::eng;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket;
    hj_job job;
    bool probe = false;  // a probe of `table` by job.S (else a join of job.R and job.S)
    hj_table table{};
    Plan plan;
    uint64_t footprint;
    size_t ws;
    Clock::time_point arrival;
};

struct Done {
    uint64_t ticket;
    hj_status status;
    double latency_s;   // arrival -> completion observed
    double queue_s;     // arrival -> admission
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<Request> reqs;
    std::vector<Clock::time_point> admitted;
    uint64_t footprint = 0;
    hj::DirectJob* h_djobs = nullptr;  // pinned, max_batch entries
    uint32_t* h_items = nullptr;       // pinned, max_items entries
    uint64_t* h_err = nullptr;         // pinned: the batch's device error word, copied back at its end
    char* ws = nullptr;                // this slot's workspace share: [error word][jobs][items][pipeline]
};

// Direct work items a slot can hold (a direct job with |S| beyond the per-job
// share of this runs through the pipeline path instead).
constexpr uint32_t kItemsPerJob = 64;

}  // namespace

struct hj_server {
    hj_server_config cfg{};
    std::vector<Slot> slots;
    size_t slot_ws = 0, slot_djobs_off = 0, slot_items_off = 0, slot_pipe_off = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request> pending;
    std::vector<Done> done;
    uint64_t next_ticket = 1;
    uint64_t used = 0;      // footprint on the device
    uint64_t inflight = 0;  // admitted, not finished
    uint64_t rejected = 0, completed = 0, batches = 0;
    bool stop = false;
    hj_status fatal = HJ_OK;
    std::thread worker;
};

namespace {

// Enqueues the slot's admitted requests on its stream.
hj_status launch_slot(hj_server* sv, Slot& s) {
    uint32_t nd = 0, items = 0;
    std::vector<size_t> piped;
    for (size_t i = 0; i < s.reqs.size(); ++i) {
        const Request& r = s.reqs[i];
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
        for (const Request& r : s.reqs)
            if (r.plan.phj && r.plan.passes == 0) cap = std::max(cap, r.plan.lds_cap);
        hj::direct_zero(d_djobs, nd, rec);
        hj::direct_join(d_djobs, d_items, items, cap, rec);
    }
    for (size_t i : piped) {
        const Request& r = s.reqs[i];
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
    while (true) {
        // retire finished batches
        bool any_busy = false;
        for (Slot& s : sv->slots) {
            if (!s.busy) continue;
            hipError_t q = hipEventQuery(s.done);
            if (q == hipErrorNotReady) {
                any_busy = true;
                continue;
            }
            const Clock::time_point now = Clock::now();
            // a set error word fails this batch's requests; the server goes on
            const bool ok = q == hipSuccess && sv->fatal == HJ_OK && *s.h_err == 0;
            for (size_t i = 0; i < s.reqs.size(); ++i) {
                Done d;
                d.ticket = s.reqs[i].ticket;
                d.status = ok ? HJ_OK : HJ_ERR_DEVICE;
                d.latency_s = std::chrono::duration<double>(now - s.reqs[i].arrival).count();
                d.queue_s = std::chrono::duration<double>(s.admitted[i] - s.reqs[i].arrival).count();
                sv->done.push_back(d);
            }
            sv->used -= s.footprint;
            sv->inflight -= s.reqs.size();
            sv->completed += s.reqs.size();
            s.reqs.clear();
            s.admitted.clear();
            s.footprint = 0;
            s.busy = false;
            if (q != hipSuccess && sv->fatal == HJ_OK) sv->fatal = HJ_ERR_DEVICE;
            sv->cv.notify_all();
        }
        // admit waiting requests into idle slots
        bool rejected_any = false;
        std::vector<Slot*> to_launch;
        for (Slot& s : sv->slots) {
            if (s.busy || sv->pending.empty()) continue;
            size_t pipe_ws = 0;
            const Clock::time_point now = Clock::now();
            while (!sv->pending.empty() && s.reqs.size() < sv->cfg.max_batch_jobs) {
                Request& r = sv->pending.front();
                if (r.footprint > sv->cfg.mem_cap_bytes || r.ws > sv->slot_ws - sv->slot_pipe_off) {
                    Done d{r.ticket, HJ_ERR_CAPACITY, 0.0, 0.0};
                    sv->done.push_back(d);
                    ++sv->rejected;
                    sv->pending.pop_front();
                    rejected_any = true;
                    continue;
                }
                if (sv->used + r.footprint > sv->cfg.mem_cap_bytes) break;  // wait for memory
                pipe_ws = std::max(pipe_ws, r.ws);
                sv->used += r.footprint;
                s.footprint += r.footprint;
                s.reqs.push_back(r);
                s.admitted.push_back(now);
                sv->pending.pop_front();
            }
            if (s.reqs.empty()) continue;
            sv->inflight += s.reqs.size();
            ++sv->batches;
            s.busy = true;
            to_launch.push_back(&s);
            any_busy = true;
        }
        // a rejection can leave nothing pending or in flight: wake drain()
        if (rejected_any) sv->cv.notify_all();
        if (!to_launch.empty()) {
            // Slots are touched by this thread only; submitters need not wait
            // for the launches.
            lk.unlock();
            hj_status st = HJ_OK;
            for (Slot* s : to_launch) {
                const hj_status e = launch_slot(sv, *s);
                if (st == HJ_OK) st = e;
            }
            lk.lock();
            if (st != HJ_OK && sv->fatal == HJ_OK) {
                sv->fatal = st;
                sv->cv.notify_all();
            }
        }
        if (sv->stop && sv->pending.empty() && !any_busy) break;
        if (any_busy) {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            sv->cv.wait_for(lk, std::chrono::microseconds(200),
                            [&] { return sv->stop || !sv->pending.empty(); });
        }
    }
}

void destroy(hj_server* sv) {
    for (Slot& s : sv->slots) {
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        if (s.h_djobs) (void)hipHostFree(s.h_djobs);
        if (s.h_items) (void)hipHostFree(s.h_items);
        if (s.h_err) (void)hipHostFree(s.h_err);
    }
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
    for (uint32_t i = 0; i < cfg->slots; ++i) {
        Slot& s = sv->slots[i];
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
    r.footprint = footprint;
    r.ws = ws_bytes_for(r.plan, job->R.n, job->S.n);
    r.arrival = Clock::now();
    {
        std::lock_guard<std::mutex> g(sv->mu);
        if (sv->fatal != HJ_OK) return fail(sv->fatal, "server stopped after a device error");
        r.ticket = sv->next_ticket++;
        *ticket = r.ticket;
        sv->pending.push_back(r);
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
    r.footprint = footprint;
    r.ws = probe_bytes_for(r.plan, table->n_r, S->n);
    r.arrival = Clock::now();
    {
        std::lock_guard<std::mutex> g(sv->mu);
        if (sv->fatal != HJ_OK) return fail(sv->fatal, "server stopped after a device error");
        r.ticket = sv->next_ticket++;
        *ticket = r.ticket;
        sv->pending.push_back(r);
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
    const uint32_t k = (uint32_t)std::min<size_t>(max, sv->done.size());
    for (uint32_t i = 0; i < k; ++i) {
        tickets[i] = sv->done[i].ticket;
        status[i] = sv->done[i].status;
        latency_s[i] = sv->done[i].latency_s;
        queue_s[i] = sv->done[i].queue_s;
    }
    sv->done.erase(sv->done.begin(), sv->done.begin() + k);
    *n = k;
    return sv->fatal;
}

hj_status hj_server_drain(hj_server* sv) {
    if (!sv) return fail(HJ_ERR_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv.wait(lk, [&] { return (sv->pending.empty() && sv->inflight == 0) || sv->fatal != HJ_OK; });
    return sv->fatal;
}

hj_status hj_server_stats(hj_server* sv, uint64_t* completed, uint64_t* rejected, uint64_t* batches,
                          uint64_t* bytes_in_use) {
    if (!sv) return fail(HJ_ERR_INVALID, "server is NULL");
    std::lock_guard<std::mutex> g(sv->mu);
    if (completed) *completed = sv->completed;
    if (rejected) *rejected = sv->rejected;
    if (batches) *batches = sv->batches;
    if (bytes_in_use) *bytes_in_use = sv->used;
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
    for (Slot& s : sv->slots)
        if (s.stream) (void)hipStreamSynchronize(s.stream);
    destroy(sv);
}

}  // extern "C"
