// Join engine shared by the single-join ABI (hj_api.cpp) and the batch
// executor (batch.cpp).  Host code only.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/hj.h"
#include "hj_internal.h"

namespace hj {
namespace eng {

constexpr size_t kAlign = 256;
constexpr uint64_t kMaxRows = 0x7FFFFFFFull;  // n < 2^31

// Thread-local error message of the last failing call.
const char* last_error();
void clear_error();
hj_status fail(hj_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

size_t align_up(size_t x);
uint64_t cdiv(uint64_t a, uint64_t b);

// Validated parameters of one join.
struct Plan {
    bool phj, one_pass;
    // non-temporal loads (kNtMinTuples): partitioning tiles, the join's S chunks
    bool nt_part, nt_s;
    uint32_t passes, b1, b2, B, P1, P2, P, tile, hash, lds_cap;
    hj_params res;  // the parameters as run (HJ_AUTO and size-dependent choices resolved)
};

// Most radix bits over all passes: 2^20 partitions keep ~4096 R tuples per
// partition (one LDS table) up to |R| = 2^31 - 1.
constexpr uint32_t kMaxRadixBits = 20;
// HJ_AUTO (costmodel.cpp): the plan with the least modelled time among SHJ,
// the direct LDS join and PHJ in one or two radix passes (and both tiles when
// p->tile is 0); keeps hash, lds_cap and flags.
void auto_params(uint64_t n_r, uint64_t n_s, hj_params* p);

// Struct Plan is below; the cost model of a plan (costmodel.cpp).
struct Plan;
double model_seconds(const Plan& pl, uint64_t n_r, uint64_t n_s, double pairs);

// Default LDS table capacity for |R| = n_r split into P partitions.
uint32_t auto_lds_cap(uint64_t n_r, uint32_t P);
hj_status check_params(const hj_params* p, uint64_t n_r, uint64_t n_s, Plan* pl);
hj_status check_call(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out, void* ws,
                     size_t ws_bytes, uint64_t* d_count, Plan* pl);
size_t ws_bytes_for(const Plan& pl, uint64_t n_r, uint64_t n_s);
// Split join (hj_build / hj_probe): build and probe workspace bytes.
size_t table_bytes_for(const Plan& pl, uint64_t n_r);
size_t probe_bytes_for(const Plan& pl, uint64_t n_r, uint64_t n_s);
// The plan a table was built with (hj_build), after checking the table's own
// fields, for a probe of n_s tuples.
hj_status table_plan(const hj_table* t, uint64_t n_s, Plan* pl);
// Enqueues the build of R's table into ws (table_bytes_for bytes).
void run_build(const Plan& pl, const hj_rel& R, void* ws, Recorder& rec);
// Enqueues a probe of table t (built with plan pl) by S.
void run_probe(const Plan& pl, const hj_table& t, const hj_rel& S, const hj_out& out, void* ws,
               uint64_t* d_count, Recorder& rec);

// Sets up the recorder of one call on `stream`: its chained scans report a
// give-up in *err, which the call's first kernel clears when `clear` (a batch
// clears its word once and runs its jobs with clear = false).  Applies the
// HJ_DEBUG_FAIL_PHASE failure injection.
void init_recorder(Recorder& rec, hipStream_t stream, uint64_t* err, bool clear);

// Enqueues one validated join on rec.stream (ws must hold ws_bytes_for bytes).
void run_join(const Plan& pl, const hj_rel& R, const hj_rel& S, const hj_out& out, void* ws,
              uint64_t* d_count, Recorder& rec);
// check_call + run_join; returns HJ_ERR_DEVICE if a launch failed.
hj_status launch_join(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out, void* ws,
                      size_t ws_bytes, uint64_t* d_count, Recorder& rec);

}  // namespace eng
}  // namespace hj
