// Batched joins: many independent joins of uneven sizes in one enqueue,
// captured once into a HIP graph and replayed.
//
// Planning (host, at plan creation):
//  * a job whose parameters say PHJ with 0 passes (R fits one LDS table) is a
//    "direct" job; all direct jobs run together in one multi-job kernel whose
//    work items are (job, S chunk), preceded by one kernel zeroing their counts;
//  * every other job runs its own SHJ/PHJ launch sequence (the single-join
//    engine) on one of kLanes streams; jobs go to lanes longest-first onto the
//    least loaded lane, and each lane reuses one workspace slice sized for its
//    largest job, so the workspace is bounded by the lanes, not the batch;
//  * without explicit per-job parameters HJ_AUTO picks them: the plan with the
//    least time under the calibrated cost model (costmodel.cpp), one-pass output.
// Running: the job table is copied from pinned host memory into the
// workspace, lanes fork from the issuing stream through events and join back
// to it.  The first run with a given workspace captures all of it (on a
// stream of the plan) into a graph; every run launches that graph on the
// caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/hj.h"
#include "engine.h"
#include "hj_internal.h"

using namespace hj::eng;

namespace {

// Concurrent lanes of the pipelined jobs.  Measured on MI355X with the
// 4096-job batch: 4 lanes 14,760 joins/s, 8 lanes 17,600-18,200, 12 lanes
// 18,900, 16 lanes 19,000, 24 lanes 18,900 (workspace grows by one lane slice
// per lane: 9.5 GB at 16).
constexpr uint32_t kLanes = 16;

struct LaneJob {
    uint32_t job;
    Plan plan;
    size_t ws;
};

}  // namespace

struct hj_batch_plan {
    uint32_t njobs = 0;
    uint32_t flags = 0;
    std::vector<hj_job> jobs;
    // direct jobs
    uint32_t ndirect = 0, direct_items = 0, direct_cap = 256;
    hj::DirectJob* h_djobs = nullptr;  // pinned staging, ndirect entries
    uint32_t* h_item_job = nullptr;    // pinned staging, direct_items entries
    size_t err_off = 0, djobs_off = 0, item_job_off = 0;
    // pipelined jobs
    std::vector<LaneJob> lane_jobs[kLanes];
    size_t lane_off[kLanes] = {0};
    size_t lane_bytes[kLanes] = {0};
    size_t ws_bytes = 0;
    // execution
    hipStream_t lane_stream[kLanes] = {nullptr};
    hipStream_t capture_stream = nullptr;  // graphs are captured here (the legacy null stream cannot capture)
    hipEvent_t fork = nullptr;
    hipEvent_t joined[kLanes] = {nullptr};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* graph_ws = nullptr;
};

namespace {

// HJ_AUTO's plan (the cost model's choice) with one-pass output.
void default_params(const hj_job& j, hj_params* p) {
    hj_default_params(p);
    p->flags = HJ_FLAG_ONE_PASS;
    auto_params(j.R.n, j.S.n, p);
}

void free_plan(hj_batch_plan* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (uint32_t l = 0; l < kLanes; ++l) {
        if (b->joined[l]) (void)hipEventDestroy(b->joined[l]);
        if (b->lane_stream[l]) (void)hipStreamDestroy(b->lane_stream[l]);
    }
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->h_djobs) (void)hipHostFree(b->h_djobs);
    if (b->h_item_job) (void)hipHostFree(b->h_item_job);
    delete b;
}

hj_status check_job(uint32_t i, const hj_job& j) {
    if (j.R.n > kMaxRows || j.S.n > kMaxRows) return fail(HJ_ERR_INVALID, "job %u: relations must have < 2^31 tuples", i);
    if (j.R.n && (!j.R.key || !j.R.rid)) return fail(HJ_ERR_INVALID, "job %u: R has tuples but a NULL array", i);
    if (j.S.n && (!j.S.key || !j.S.rid)) return fail(HJ_ERR_INVALID, "job %u: S has tuples but a NULL array", i);
    if (j.out.capacity && (!j.out.rid_r || !j.out.rid_s))
        return fail(HJ_ERR_INVALID, "job %u: out has capacity but a NULL array", i);
    if (!j.d_count) return fail(HJ_ERR_INVALID, "job %u: d_count is NULL", i);
    return HJ_OK;
}

// Enqueues the whole batch on `stream` (lanes fork from and join back to it).
hj_status enqueue(hj_batch_plan* b, char* ws, hipStream_t stream) {
    hipError_t e = hipSuccess;
    uint64_t* err = (uint64_t*)(ws + b->err_off);  // one error word for the whole batch
    hj::DirectJob* d_djobs = (hj::DirectJob*)(ws + b->djobs_off);
    uint32_t* d_item_job = (uint32_t*)(ws + b->item_job_off);
    if (b->ndirect) {
        e = hipMemcpyAsync(d_djobs, b->h_djobs, sizeof(hj::DirectJob) * b->ndirect, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess && b->direct_items)
            e = hipMemcpyAsync(d_item_job, b->h_item_job, sizeof(uint32_t) * b->direct_items,
                               hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return fail(HJ_ERR_DEVICE, "job table upload failed: %s", hipGetErrorString(e));
    }
    hj::Recorder main_rec;
    init_recorder(main_rec, stream, err, false);
    // cleared before the lanes fork, so no job's report can be lost
    hj::zero_pair(err, nullptr, main_rec);
    bool any_lane = false;
    for (uint32_t l = 0; l < kLanes; ++l) any_lane |= !b->lane_jobs[l].empty();
    if (any_lane) {
        e = hipEventRecord(b->fork, stream);
        for (uint32_t l = 0; e == hipSuccess && l < kLanes; ++l)
            if (!b->lane_jobs[l].empty()) e = hipStreamWaitEvent(b->lane_stream[l], b->fork, 0);
        if (e != hipSuccess) return fail(HJ_ERR_DEVICE, "lane fork failed: %s", hipGetErrorString(e));
    }
    hj::direct_zero(d_djobs, b->ndirect, main_rec);
    hj::direct_join(d_djobs, d_item_job, b->direct_items, b->direct_cap, main_rec);
    if (main_rec.err != hipSuccess) return fail(HJ_ERR_DEVICE, "launch failed: %s", hipGetErrorString(main_rec.err));
    for (uint32_t l = 0; l < kLanes; ++l) {
        if (b->lane_jobs[l].empty()) continue;
        hj::Recorder rec;
        init_recorder(rec, b->lane_stream[l], err, false);
        for (const LaneJob& lj : b->lane_jobs[l]) {
            const hj_job& j = b->jobs[lj.job];
            run_join(lj.plan, j.R, j.S, j.out, ws + b->lane_off[l], j.d_count, rec);
        }
        if (rec.err != hipSuccess) return fail(HJ_ERR_DEVICE, "launch failed: %s", hipGetErrorString(rec.err));
        e = hipEventRecord(b->joined[l], b->lane_stream[l]);
        if (e == hipSuccess) e = hipStreamWaitEvent(stream, b->joined[l], 0);
        if (e != hipSuccess) return fail(HJ_ERR_DEVICE, "lane join failed: %s", hipGetErrorString(e));
    }
    return HJ_OK;
}

}  // namespace

namespace {
// Plans the batch; sizing_only: stops after the workspace layout (no pinned
// staging, streams or events).
hj_status create_plan(uint32_t njobs, const hj_job* jobs, const hj_params* params, uint32_t flags,
                      bool sizing_only, hj_batch_plan** plan);
}  // namespace

extern "C" {

hj_status hj_batch_plan_create(uint32_t njobs, const hj_job* jobs, const hj_params* params, uint32_t flags,
                               hj_batch_plan** plan) {
    return create_plan(njobs, jobs, params, flags, false, plan);
}

size_t hj_batch_bytes(uint32_t njobs, const hj_job* jobs, const hj_params* params) {
    hj_batch_plan* b = nullptr;
    if (create_plan(njobs, jobs, params, HJ_BATCH_NO_GRAPH, true, &b) != HJ_OK) return 0;
    const size_t n = b->ws_bytes;
    free_plan(b);
    clear_error();
    return n;
}

hj_status hj_batch(uint32_t njobs, const hj_job* jobs, const hj_params* params, void* ws, size_t ws_bytes,
                   void* stream) {
    hj_batch_plan* b = nullptr;
    hj_status st = create_plan(njobs, jobs, params, HJ_BATCH_NO_GRAPH, false, &b);
    if (st != HJ_OK) return st;
    st = hj_batch_run(b, ws, ws_bytes, stream);
    // the job table is copied from the plan's pinned staging: wait before freeing it
    const hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    free_plan(b);
    if (st != HJ_OK) return st;
    if (e != hipSuccess) return fail(HJ_ERR_DEVICE, "batch failed: %s", hipGetErrorString(e));
    clear_error();
    return HJ_OK;
}

}  // extern "C"

namespace {

hj_status create_plan(uint32_t njobs, const hj_job* jobs, const hj_params* params, uint32_t flags,
                      bool sizing_only, hj_batch_plan** plan) {
    if (!plan) return fail(HJ_ERR_INVALID, "plan is NULL");
    *plan = nullptr;
    if (njobs && !jobs) return fail(HJ_ERR_INVALID, "jobs is NULL");
    if (flags & ~HJ_BATCH_NO_GRAPH) return fail(HJ_ERR_INVALID, "unknown batch flags 0x%x", flags);
    hj_batch_plan* b = new (std::nothrow) hj_batch_plan;
    if (!b) return fail(HJ_ERR_DEVICE, "out of host memory");
    b->njobs = njobs;
    b->flags = flags;
    b->jobs.assign(jobs, jobs + njobs);
    std::vector<uint32_t> direct;
    std::vector<LaneJob> piped;
    for (uint32_t i = 0; i < njobs; ++i) {
        const hj_job& j = jobs[i];
        hj_status st = check_job(i, j);
        if (st != HJ_OK) {
            free_plan(b);
            return st;
        }
        hj_params p;
        if (params) p = params[i]; else default_params(j, &p);
        Plan pl;
        st = check_params(&p, j.R.n, j.S.n, &pl);
        if (st != HJ_OK) {
            free_plan(b);
            return fail(st, "job %u: %s", i, last_error());
        }
        if (pl.phj && pl.passes == 0) {
            direct.push_back(i);
            b->direct_cap = std::max(b->direct_cap, pl.lds_cap);
        } else {
            piped.push_back(LaneJob{i, pl, ws_bytes_for(pl, j.R.n, j.S.n)});
        }
    }
    // direct jobs: descriptors and the item -> job map
    b->ndirect = (uint32_t)direct.size();
    uint64_t items = 0;
    for (uint32_t i : direct)
        if (jobs[i].R.n && jobs[i].S.n) items += cdiv(jobs[i].S.n, hj::kJoinChunk);
    if (items > 0x7FFFFFFFull) {
        free_plan(b);
        return fail(HJ_ERR_INVALID, "too many direct work items");
    }
    b->direct_items = (uint32_t)items;
    if (b->ndirect && !sizing_only) {
        hipError_t e = hipHostMalloc((void**)&b->h_djobs, sizeof(hj::DirectJob) * b->ndirect, hipHostMallocDefault);
        if (e == hipSuccess && b->direct_items)
            e = hipHostMalloc((void**)&b->h_item_job, sizeof(uint32_t) * b->direct_items, hipHostMallocDefault);
        if (e != hipSuccess) {
            free_plan(b);
            return fail(HJ_ERR_DEVICE, "pinned staging allocation failed: %s", hipGetErrorString(e));
        }
        uint32_t item = 0;
        for (uint32_t d = 0; d < b->ndirect; ++d) {
            const hj_job& j = jobs[direct[d]];
            hj::DirectJob& dj = b->h_djobs[d];
            std::memset(&dj, 0, sizeof dj);
            dj.rk = j.R.key;
            dj.rr = j.R.rid;
            dj.sk = j.S.key;
            dj.sr = j.S.rid;
            dj.out_r = j.out.rid_r;
            dj.out_s = j.out.rid_s;
            dj.capacity = j.out.capacity;
            dj.count = j.d_count;
            dj.n_r = (uint32_t)j.R.n;
            dj.n_s = (uint32_t)j.S.n;
            dj.item0 = item;
            const uint32_t n_items = (j.R.n && j.S.n) ? (uint32_t)cdiv(j.S.n, hj::kJoinChunk) : 0u;
            for (uint32_t k = 0; k < n_items; ++k) b->h_item_job[item + k] = d;
            item += n_items;
        }
    }
    // pipelined jobs: longest first onto the least loaded lane
    std::sort(piped.begin(), piped.end(), [&](const LaneJob& x, const LaneJob& y) {
        const uint64_t a = jobs[x.job].R.n + jobs[x.job].S.n, c = jobs[y.job].R.n + jobs[y.job].S.n;
        return a != c ? a > c : x.job < y.job;
    });
    uint64_t load[kLanes] = {0};
    for (const LaneJob& lj : piped) {
        uint32_t best = 0;
        for (uint32_t l = 1; l < kLanes; ++l)
            if (load[l] < load[best]) best = l;
        load[best] += jobs[lj.job].R.n + jobs[lj.job].S.n + 65536;  // + fixed cost of a launch sequence
        b->lane_jobs[best].push_back(lj);
        b->lane_bytes[best] = std::max(b->lane_bytes[best], lj.ws);
    }
    // workspace: [error word][direct jobs][item map][lane 0]...[lane 15]
    size_t off = 0;
    b->err_off = off;
    off += align_up(sizeof(uint64_t));
    b->djobs_off = off;
    off += align_up(sizeof(hj::DirectJob) * std::max<uint32_t>(b->ndirect, 1));
    b->item_job_off = off;
    off += align_up(sizeof(uint32_t) * std::max<uint32_t>(b->direct_items, 1));
    for (uint32_t l = 0; l < kLanes; ++l) {
        b->lane_off[l] = off;
        off += align_up(b->lane_bytes[l]);
    }
    b->ws_bytes = off;
    if (sizing_only) {
        *plan = b;
        return HJ_OK;
    }
    // lane streams and events (default priority)
    hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
    for (uint32_t l = 0; e == hipSuccess && l < kLanes; ++l) {
        e = hipStreamCreateWithFlags(&b->lane_stream[l], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->joined[l], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        free_plan(b);
        return fail(HJ_ERR_DEVICE, "stream/event creation failed: %s", hipGetErrorString(e));
    }
    *plan = b;
    clear_error();
    return HJ_OK;
}

}  // namespace

extern "C" {

size_t hj_batch_workspace_bytes(const hj_batch_plan* plan) { return plan ? plan->ws_bytes : 0; }

uint32_t hj_batch_direct_jobs(const hj_batch_plan* plan) { return plan ? plan->ndirect : 0; }

size_t hj_batch_graph_nodes(const hj_batch_plan* plan) {
    if (!plan || !plan->graph) return 0;
    size_t n = 0;
    return hipGraphGetNodes(plan->graph, nullptr, &n) == hipSuccess ? n : 0;
}

hj_status hj_batch_run(hj_batch_plan* b, void* ws, size_t ws_bytes, void* stream) {
    if (!b) return fail(HJ_ERR_INVALID, "plan is NULL");
    if (!ws || ws_bytes < b->ws_bytes)
        return fail(HJ_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", b->ws_bytes, ws ? ws_bytes : 0);
    if ((uintptr_t)ws % kAlign) return fail(HJ_ERR_INVALID, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    if (b->flags & HJ_BATCH_NO_GRAPH) return enqueue(b, (char*)ws, s);
    if (!b->exec || b->graph_ws != ws) {
        if (b->exec) {
            (void)hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
        if (b->graph) {
            (void)hipGraphDestroy(b->graph);
            b->graph = nullptr;
        }
        hipStream_t cs = b->capture_stream;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return fail(HJ_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        hj_status st = enqueue(b, (char*)ws, cs);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        if (st != HJ_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return fail(HJ_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return fail(HJ_ERR_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
        }
        b->graph = g;
        b->graph_ws = ws;
    }
    hipError_t e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return fail(HJ_ERR_DEVICE, "graph launch failed: %s", hipGetErrorString(e));
    clear_error();
    return HJ_OK;
}

void hj_batch_plan_destroy(hj_batch_plan* plan) { free_plan(plan); }

}  // extern "C"
