// Admission and retirement of a join server's requests, apart from the device.
//
// Requests wait in one FIFO, each with a footprint (the device bytes it holds
// while it runs) and a workspace need.  `slots` slots each run one batch at a
// time.  admit() fills every idle slot from the head of the FIFO: a request
// whose footprint alone exceeds the memory cap, or whose workspace exceeds a
// slot's share, is rejected; otherwise requests join the slot's batch while
// the footprints of everything admitted stay within the cap and the batch
// within max_batch requests, and the first one that does not fit stops the
// admission (first come, first served: nothing overtakes it).  retire() ends
// a slot's batch and records each request's latency (arrival -> retirement)
// and queueing time (arrival -> admission).
//
// The core holds no device state and no clock: callers pass the time (seconds
// on any clock) and run the batches themselves (the server on HIP streams, a
// test on a simulated device with a virtual clock).
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <vector>

#include "../../include/hj.h"

namespace hj {
namespace srv {

struct CoreConfig {
    uint32_t slots;
    uint32_t max_batch;
    uint64_t mem_cap;
    size_t slot_ws;  // workspace a slot's batch can give one request
};

struct Finished {
    uint64_t ticket;
    hj_status status;
    double latency_s;  // arrival -> retirement
    double queue_s;    // arrival -> admission
};

template <class Payload>
struct Core {
    struct Req {
        uint64_t ticket;
        uint64_t footprint;
        size_t ws;
        double arrival;
        Payload payload;
    };
    struct Slot {
        bool busy = false;
        std::vector<Req> reqs;
        std::vector<double> admitted;
        uint64_t footprint = 0;
    };

    CoreConfig cfg;
    std::vector<Slot> slots;
    std::deque<Req> pending;
    std::vector<Finished> done;
    uint64_t next_ticket = 1;
    uint64_t used = 0;      // footprint of the admitted requests
    uint64_t inflight = 0;  // admitted, not retired
    uint64_t rejected = 0, completed = 0, batches = 0;

    explicit Core(const CoreConfig& c) : cfg(c), slots(c.slots) {}

    uint64_t submit(uint64_t footprint, size_t ws, double now, const Payload& p) {
        const uint64_t t = next_ticket++;
        pending.push_back(Req{t, footprint, ws, now, p});
        return t;
    }

    // Fills the idle slots; returns the slots whose batches are to be launched.
    // *rejected_any tells whether a request was turned away.
    std::vector<uint32_t> admit(double now, bool* rejected_any) {
        std::vector<uint32_t> launch;
        *rejected_any = false;
        for (uint32_t i = 0; i < slots.size(); ++i) {
            Slot& s = slots[i];
            if (s.busy || pending.empty()) continue;
            while (!pending.empty() && s.reqs.size() < cfg.max_batch) {
                Req& r = pending.front();
                if (r.footprint > cfg.mem_cap || r.ws > cfg.slot_ws) {
                    done.push_back(Finished{r.ticket, HJ_ERR_CAPACITY, 0.0, 0.0});
                    ++rejected;
                    pending.pop_front();
                    *rejected_any = true;
                    continue;
                }
                if (used + r.footprint > cfg.mem_cap) break;  // wait for memory
                used += r.footprint;
                s.footprint += r.footprint;
                s.reqs.push_back(r);
                s.admitted.push_back(now);
                pending.pop_front();
            }
            if (s.reqs.empty()) continue;
            inflight += s.reqs.size();
            ++batches;
            s.busy = true;
            launch.push_back(i);
        }
        return launch;
    }

    // Ends slot i's batch: every request finishes with HJ_OK if ok, else with
    // fail_status; the slot's footprint is released.
    void retire(uint32_t i, bool ok, double now, hj_status fail_status) {
        Slot& s = slots[i];
        for (size_t k = 0; k < s.reqs.size(); ++k)
            done.push_back(Finished{s.reqs[k].ticket, ok ? HJ_OK : fail_status, now - s.reqs[k].arrival,
                                    s.admitted[k] - s.reqs[k].arrival});
        used -= s.footprint;
        inflight -= s.reqs.size();
        completed += s.reqs.size();
        s.reqs.clear();
        s.admitted.clear();
        s.footprint = 0;
        s.busy = false;
    }

    bool idle() const { return pending.empty() && inflight == 0; }
};

// The least footprint a request can have: its relations and output arrays
// (8 bytes a tuple or a pair), its count and its workspace.  The server
// admits by the larger of this and what the caller declares.
inline uint64_t least_footprint(uint64_t n_r, uint64_t n_s, uint64_t capacity, size_t ws) {
    return 8 * (n_r + n_s) + 8 * capacity + sizeof(uint64_t) + ws;
}

}  // namespace srv
}  // namespace hj
