// The join server's admission core (csrc/server_core.h) on a simulated device
// with a virtual clock: requests arrive by a seeded random process, a slot's
// batch runs for a modelled time (a fixed launch cost plus a cost per request),
// and an event loop advances the clock from event to event.  Checked after
// every step:
//   * the admitted footprints never exceed the cap and always equal the sum
//     over the busy slots;
//   * no batch exceeds max_batch; admission is first come, first served (the
//     admitted tickets rise across all slots);
//   * work is conserved: after admission, either nothing waits, or no slot is
//     idle, or the head of the queue does not fit the memory left;
//   * every request finishes exactly once, rejected exactly when its own
//     footprint exceeds the cap or its workspace a slot's share;
//   * latency = retirement - arrival, queueing = admission - arrival, both >= 0;
// and, with one slot and batches of one, the finish times equal a FIFO
// single-server queue computed directly.
// Built with g++ -fsanitize=address,undefined by tests/test_host_sanitized.py.
#include <cassert>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <queue>
#include <random>
#include <set>
#include <vector>

#include "server_core.h"

using hj::srv::Core;
using hj::srv::CoreConfig;

namespace {

int failures = 0;
#define CHECK(c)                                                                   \
    do {                                                                           \
        if (!(c)) {                                                                \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                            \
        }                                                                          \
    } while (0)

struct Payload {
    uint64_t id;
};

struct Arrival {
    double t;
    uint64_t footprint;
    size_t ws;
};

struct Outcome {
    hj_status status;
    double latency, queue;
};

// Runs the arrivals through a core on a simulated device; returns each
// request's outcome by ticket (tickets are issued in arrival order from 1).
std::map<uint64_t, Outcome> simulate(const CoreConfig& cfg, const std::vector<Arrival>& arr, double launch_s,
                                     double per_req_s, uint64_t* batches_out) {
    Core<Payload> c(cfg);
    std::vector<double> busy_until(cfg.slots, 0.0);
    std::map<uint64_t, Outcome> out;
    uint64_t last_admitted = 0;
    size_t next = 0;
    double now = 0.0;
    while (next < arr.size() || !c.idle()) {
        // retire the batches that end by now
        for (uint32_t i = 0; i < cfg.slots; ++i)
            if (c.slots[i].busy && busy_until[i] <= now) c.retire(i, true, now, HJ_ERR_DEVICE);
        // arrivals up to now
        while (next < arr.size() && arr[next].t <= now) {
            const uint64_t t = c.submit(arr[next].footprint, arr[next].ws, arr[next].t, Payload{next});
            CHECK(t == next + 1);
            ++next;
        }
        bool rej = false;
        const std::vector<uint32_t> launch = c.admit(now, &rej);
        for (uint32_t i : launch) {
            const auto& s = c.slots[i];
            CHECK(s.busy);
            CHECK(!s.reqs.empty() && s.reqs.size() <= cfg.max_batch);
            for (const auto& r : s.reqs) {
                CHECK(r.ticket > last_admitted);  // first come, first served
                last_admitted = r.ticket;
            }
            busy_until[i] = now + launch_s + per_req_s * (double)s.reqs.size();
        }
        // invariants
        uint64_t sum = 0;
        uint32_t idle = 0;
        for (const auto& s : c.slots) {
            sum += s.footprint;
            idle += s.busy ? 0u : 1u;
        }
        CHECK(sum == c.used);
        CHECK(c.used <= cfg.mem_cap);
        if (!c.pending.empty() && idle > 0) CHECK(c.used + c.pending.front().footprint > cfg.mem_cap);
        // collect what finished
        for (const auto& f : c.done) {
            CHECK(out.find(f.ticket) == out.end());
            out[f.ticket] = Outcome{f.status, f.latency_s, f.queue_s};
        }
        c.done.clear();
        // next event: an arrival or a batch end
        double t_next = INFINITY;
        if (next < arr.size()) t_next = arr[next].t;
        for (uint32_t i = 0; i < cfg.slots; ++i)
            if (c.slots[i].busy) t_next = std::min(t_next, busy_until[i]);
        if (t_next == INFINITY) break;
        now = std::max(now, t_next);
    }
    CHECK(c.idle());
    CHECK(c.used == 0);
    *batches_out = c.batches;
    return out;
}

void random_workloads() {
    std::mt19937_64 rng(20240611);
    for (int trial = 0; trial < 200; ++trial) {
        CoreConfig cfg;
        cfg.slots = 1 + (uint32_t)(rng() % 16);
        cfg.max_batch = 1 + (uint32_t)(rng() % 64);
        cfg.mem_cap = 1000 + rng() % 100000;
        cfg.slot_ws = 100 + rng() % 10000;
        const size_t n = 50 + rng() % 2000;
        std::vector<Arrival> arr;
        double t = 0.0;
        std::exponential_distribution<double> gap(1.0 / (1e-5 + 1e-4 * (double)(rng() % 10)));
        for (size_t i = 0; i < n; ++i) {
            t += gap(rng);
            // mostly fitting requests, a few that exceed the cap or a slot
            const uint64_t fp = (rng() % 50 == 0) ? cfg.mem_cap + 1 + rng() % 100 : 1 + rng() % (cfg.mem_cap / 4 + 1);
            const size_t ws = (rng() % 60 == 0) ? cfg.slot_ws + 1 : rng() % (cfg.slot_ws + 1);
            arr.push_back(Arrival{t, fp, ws});
        }
        uint64_t batches = 0;
        const auto out = simulate(cfg, arr, 2e-5, 5e-6, &batches);
        CHECK(out.size() == n);
        uint64_t ok = 0;
        for (size_t i = 0; i < n; ++i) {
            const auto it = out.find(i + 1);
            if (it == out.end()) {
                CHECK(false);
                continue;
            }
            const bool too_big = arr[i].footprint > cfg.mem_cap || arr[i].ws > cfg.slot_ws;
            CHECK((it->second.status == HJ_ERR_CAPACITY) == too_big);
            if (!too_big) {
                CHECK(it->second.status == HJ_OK);
                CHECK(it->second.queue >= 0.0);
                CHECK(it->second.latency >= it->second.queue);
                ++ok;
            }
        }
        CHECK(batches <= ok);
    }
}

// One slot, batches of one: a FIFO single-server queue.  Request i starts at
// max(its arrival, the previous finish) and takes launch + per_req.
void single_server_closed_form() {
    CoreConfig cfg{1, 1, 1u << 30, 1u << 20};
    std::mt19937_64 rng(7);
    std::exponential_distribution<double> gap(1.0 / 3e-5);
    std::vector<Arrival> arr;
    double t = 0.0;
    for (int i = 0; i < 5000; ++i) {
        t += gap(rng);
        arr.push_back(Arrival{t, 1 + rng() % 1000, rng() % 1000});
    }
    const double launch = 2e-5, per = 5e-6;
    uint64_t batches = 0;
    const auto out = simulate(cfg, arr, launch, per, &batches);
    CHECK(batches == arr.size());
    double free_at = 0.0;
    for (size_t i = 0; i < arr.size(); ++i) {
        // the simulated server admits at the first event at or after both the
        // arrival and the previous finish
        const double start = std::max(arr[i].t, free_at);
        const double finish = start + launch + per;
        const Outcome& o = out.at(i + 1);
        CHECK(std::fabs(o.queue - (start - arr[i].t)) < 1e-9);
        CHECK(std::fabs(o.latency - (finish - arr[i].t)) < 1e-9);
        free_at = finish;
    }
}

// The memory cap orders admission: with a cap of two requests and four slots,
// at most two run at once, and the third waits for a retirement even though
// slots are idle.
void cap_blocks_admission() {
    CoreConfig cfg{4, 8, 200, 1000};
    Core<Payload> c(cfg);
    for (int i = 0; i < 3; ++i) c.submit(100, 10, 0.0, Payload{(uint64_t)i});
    bool rej = false;
    auto l = c.admit(0.0, &rej);
    CHECK(l.size() == 1 && c.slots[l[0]].reqs.size() == 2);  // one batch of two: the cap is reached
    CHECK(c.pending.size() == 1 && c.used == 200);
    l = c.admit(0.5, &rej);
    CHECK(l.empty());
    c.retire(0, true, 1.0, HJ_ERR_DEVICE);
    CHECK(c.used == 0 && c.done.size() == 2);
    l = c.admit(1.0, &rej);
    CHECK(l.size() == 1 && c.slots[l[0]].reqs.size() == 1 && c.slots[l[0]].reqs[0].ticket == 3);
    c.retire(l[0], false, 2.0, HJ_ERR_DEVICE);
    CHECK(c.done.back().status == HJ_ERR_DEVICE && c.done.back().queue_s == 1.0 && c.done.back().latency_s == 2.0);
    CHECK(c.idle());
}

void least_footprint() {
    CHECK(hj::srv::least_footprint(10, 20, 30, 1000) == 8 * 30 + 8 * 30 + 8 + 1000);
    CHECK(hj::srv::least_footprint(0, 0, 0, 0) == 8);
}

}  // namespace

int main() {
    random_workloads();
    single_server_closed_form();
    cap_blocks_admission();
    least_footprint();
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("server core: all checks passed\n");
    return 0;
}
