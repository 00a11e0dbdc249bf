// Join engine: argument validation, workspace layouts and the launch
// sequences of the simple (SHJ, Algorithm 1) and radix-partitioned (PHJ,
// Algorithm 2) hash joins, shared by the single-join ABI and the batch
// executor.
//
// SHJ: fill table -> build -> count -> scan -> write (or build -> one-pass write).
// PHJ: per pass: hist -> scan -> scatter (R and S in the same launches); then
// plan the partition pairs -> HBM tables for oversized R partitions -> count ->
// scan -> write (or one-pass write).
// Everything is enqueued on one stream; no host synchronisation, no
// host<->device copy and no allocation happen here.
#include "engine.h"
#include "hj_side.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <string>

namespace hj {
namespace eng {

namespace {
thread_local std::string g_err;
}  // namespace

const char* last_error() { return g_err.c_str(); }
void clear_error() { g_err.clear(); }

hj_status fail(hj_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

uint32_t ceil_log2(uint64_t v) {
    uint32_t l = 0;
    while ((1ull << l) < v) ++l;
    return l;
}

uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Bump-carves aligned sub-buffers out of one workspace.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <typename T>
    T* take(uint64_t count) {
        T* p = base ? (T*)(base + off) : nullptr;
        off += align_up(sizeof(T) * (size_t)std::max<uint64_t>(count, 1));
        return p;
    }
};


// LDS per CU on gfx950, and what a join workgroup takes beyond its dynamic
// tables (static LDS plus allocation rounding; measured: a 54,080-byte table
// set no longer fits three workgroups per CU, 53,312 bytes does).
constexpr size_t kLdsPerCu = 160 * 1024;
constexpr size_t kJoinStaticLds = 1024;

uint32_t join_blocks_per_cu(uint32_t cap) {
    return (uint32_t)(kLdsPerCu / (hj::join_lds_bytes(cap, true) + kJoinStaticLds));
}

// Default LDS table capacity: room for a partition three standard deviations
// above the mean size (uniform hashing), then grown to the largest capacity
// that keeps the same number of write-kernel workgroups per CU and the same
// build kernel (registers per thread grow with the build's tuples per thread).
uint32_t auto_lds_cap(uint64_t n_r, uint32_t P) {
    const double avg = std::ceil((double)n_r / (double)P);
    const double need = avg + 3.0 * std::sqrt(avg) + 32.0;
    uint32_t cap = (uint32_t)std::min<double>(hj::kMaxLdsCap, std::max(256.0, need));
    cap = (cap + 63) / 64 * 64;
    if (cap > hj::kMaxLdsCap) cap = hj::kMaxLdsCap;
    const uint32_t bpc = join_blocks_per_cu(cap);
    while (cap + 64 <= hj::kMaxLdsCap && join_blocks_per_cu(cap + 64) == bpc &&
           hj::join_rpt(cap + 64) == hj::join_rpt(cap))
        cap += 64;
    return cap;
}

namespace {
// The parameters a plan runs with, every size-dependent choice filled in.
void fill_resolved(const hj_params* p, Plan* pl) {
    hj_params& r = pl->res;
    r = *p;
    r.algo = pl->phj ? HJ_PHJ : HJ_SHJ;
    r.tile = pl->tile;
    if (!pl->phj) return;
    r.passes = pl->passes;
    r.bits[0] = pl->b1;
    r.bits[1] = pl->b2;
    r.lds_cap = pl->lds_cap;
    if (pl->one_pass) r.flags |= HJ_FLAG_ONE_PASS;
}
}  // namespace

hj_status check_params(const hj_params* p, uint64_t n_r, uint64_t n_s, Plan* pl) {
    if (!p) return fail(HJ_ERR_INVALID, "params is NULL");
    if (p->algo == HJ_AUTO) {
        hj_params q = *p;
        auto_params(n_r, n_s, &q);
        return check_params(&q, n_r, n_s, pl);
    }
    if (p->flags & ~HJ_FLAG_ONE_PASS) return fail(HJ_ERR_INVALID, "unknown flags 0x%x", p->flags);
    if (p->algo != HJ_SHJ && p->algo != HJ_PHJ) return fail(HJ_ERR_INVALID, "unknown algo %u", p->algo);
    if (p->hash != HJ_HASH_IDENTITY && p->hash != HJ_HASH_MURMUR2)
        return fail(HJ_ERR_INVALID, "unknown hash %u", p->hash);
    if (p->tile != 0 && p->tile != 1024 && p->tile != 2048 && p->tile != 4096 && p->tile != 8192)
        return fail(HJ_ERR_INVALID, "tile must be 0 or a power of two in 1024..8192 (got %u)", p->tile);
    pl->phj = p->algo == HJ_PHJ;
    pl->one_pass = (p->flags & HJ_FLAG_ONE_PASS) != 0;
    pl->tile = p->tile ? p->tile : 4096;  // PHJ with partitioning: chosen below
    pl->hash = p->hash;
    pl->passes = 0;
    pl->b1 = pl->b2 = pl->B = 0;
    pl->P1 = pl->P2 = pl->P = 1;
    pl->lds_cap = 0;
    pl->nt_part = n_r + n_s >= hj::kNtMinTuples;
    pl->nt_s = pl->nt_part && n_s <= 2 * n_r;
    if (!pl->phj) {
        fill_resolved(p, pl);
        return HJ_OK;
    }
    if (p->passes == 0) {
        // no partitioning: R must fit one LDS table
        if (n_r > hj::kMaxLdsCap)
            return fail(HJ_ERR_INVALID, "passes 0 needs |R| <= %u (got %llu)", hj::kMaxLdsCap,
                        (unsigned long long)n_r);
        pl->passes = 0;
        pl->one_pass = true;
        const uint32_t need = (uint32_t)std::max<uint64_t>(256, (n_r + 63) / 64 * 64);
        pl->lds_cap = p->lds_cap ? std::max(p->lds_cap, need) : need;
        if (pl->lds_cap > hj::kMaxLdsCap) return fail(HJ_ERR_INVALID, "lds_cap above %u", hj::kMaxLdsCap);
        fill_resolved(p, pl);
        return HJ_OK;
    }
    if (p->passes != 1 && p->passes != 2)
        return fail(HJ_ERR_INVALID, "passes must be 0, 1 or 2 (got %u)", p->passes);
    pl->passes = p->passes;
    pl->b1 = p->bits[0];
    pl->b2 = p->passes == 2 ? p->bits[1] : 0;
    if (pl->b1 < 1 || pl->b1 > 13) return fail(HJ_ERR_INVALID, "bits[0] must be in 1..13 (got %u)", pl->b1);
    if (p->passes == 2 && (pl->b2 < 1 || pl->b2 > 13))
        return fail(HJ_ERR_INVALID, "bits[1] must be in 1..13 (got %u)", pl->b2);
    pl->B = pl->b1 + pl->b2;
    if (pl->B > kMaxRadixBits)
        return fail(HJ_ERR_INVALID, "total radix bits must be <= %u (got %u)", kMaxRadixBits, pl->B);
    pl->P1 = 1u << pl->b1;
    pl->P2 = 1u << pl->b2;
    pl->P = 1u << pl->B;
    if (p->lds_cap) {
        if (p->lds_cap % 64 || p->lds_cap < 256 || p->lds_cap > 8192)
            return fail(HJ_ERR_INVALID, "lds_cap must be 0 or a multiple of 64 in 256..8192 (got %u)",
                        p->lds_cap);
        pl->lds_cap = p->lds_cap;
    } else {
        pl->lds_cap = auto_lds_cap(n_r, pl->P);
    }
    if (!p->tile) pl->tile = hj::default_tile(n_r, n_s, pl->passes, pl->b1);
    fill_resolved(p, pl);
    return HJ_OK;
}

// Every workspace layout starts with the call's error word (kErrLookback;
// hj_workspace_status reads it), then its own buffers.
// Workspace layout; with base == nullptr only the size is computed.
struct PhjWs {
    uint64_t* err;
    hj::PartSeg* segs1;
    uint32_t* tb1;
    uint32_t* hist1;
    int32_t *keyA, *ridA;
    hj::PartSeg* segs2;
    uint32_t* tb2;
    uint32_t* tseg2;
    uint32_t* hist2;     // pass-2 histogram (not counted)
    uint8_t* rows;       // pass-1 count rows (counted pass 2)
    uint32_t* esc;       //   and their escapes
    uint32_t* tot2;      // counted pass 2: final partition totals (zeroed block)
    uint32_t* cur2;      //   and reservation cursors (zeroed block)
    int32_t *keyB, *ridB;
    hj::PartPair* pairs;
    uint32_t* item_begin;
    uint32_t* ovf_begin;
    hj::ItemRec* item_rec;
    uint32_t* ovf_part;
    uint64_t* wave_cnt;
    uint64_t* ovf_table;
    uint32_t* ovf_next;
    hj::HeavyQueue* heavy;  // one-pass heavy-tuple queue (cleared with the scan states)
    hj::HotKeys* hot;       // hot keys of the HBM-table build (cleared with the scan states)
    uint64_t* st1;     // scan states (cleared by the first kernel): pass-1 histogram,
    uint64_t* st2;     //   pass-2 histogram,
    uint64_t* stw;     //   per-wave match counts,
    uint64_t* stp;     //   join plan
    uint64_t* zero;    // the queue and the scan states, cleared by the first kernel
    uint64_t nzero;    // words from `zero` on to clear
    uint64_t tiles1, tiles2_ub, items_ub, ovf_ub;
    size_t bytes;
};

// n_r, n_s: tuples partitioned by this call (either may be 0 for a table
// build or a probe); n_r_tab: tuples of the R that is joined (sizes the HBM
// tables of oversized R partitions).
PhjWs phj_layout(const Plan& pl, uint64_t n_r, uint64_t n_s, uint64_t n_r_tab, void* base) {
    PhjWs w{};
    Carver c(base);
    const uint64_t n = n_r + n_s;
    w.tiles1 = cdiv(n_r, pl.tile) + cdiv(n_s, pl.tile);
    w.err = c.take<uint64_t>(1);
    w.segs1 = c.take<hj::PartSeg>(2);
    w.tb1 = c.take<uint32_t>(3);
    w.hist1 = c.take<uint32_t>(w.tiles1 * pl.P1);
    w.keyA = c.take<int32_t>(n);
    w.ridA = c.take<int32_t>(n);
    const bool counted = hj::counted_pass2(pl.passes, pl.b1, pl.b2);
    if (pl.passes == 2) {
        w.tiles2_ub = cdiv(n, pl.tile) + 2ull * pl.P1;
        w.segs2 = c.take<hj::PartSeg>(2ull * pl.P1);
        w.tb2 = c.take<uint32_t>(2ull * pl.P1 + 1);
        w.tseg2 = c.take<uint32_t>(w.tiles2_ub);
        if (counted) {
            w.rows = c.take<uint8_t>(w.tiles1 * pl.P);
            w.esc = c.take<uint32_t>(w.tiles1 * hj::kCountEsc);
        } else {
            w.hist2 = c.take<uint32_t>(w.tiles2_ub * pl.P2);
        }
        w.keyB = c.take<int32_t>(n);
        w.ridB = c.take<int32_t>(n);
    }
    w.pairs = c.take<hj::PartPair>(pl.P);
    w.item_begin = c.take<uint32_t>(pl.P + 1ull);
    w.ovf_begin = c.take<uint32_t>(pl.P + 1ull);
    w.items_ub = hj::join_grid(pl.P, n_s);
    w.ovf_ub = hj::ovf_grid(pl.P, n_r_tab);
    w.item_rec = c.take<hj::ItemRec>(w.items_ub);
    w.ovf_part = c.take<uint32_t>(w.ovf_ub);
    w.wave_cnt = c.take<uint64_t>(w.items_ub * hj::kJoinWaves);
    w.ovf_table = c.take<uint64_t>(2 * n_r_tab);
    w.ovf_next = c.take<uint32_t>(n_r_tab);
    const uint64_t n1 = hj::scan_state_words(w.tiles1 * pl.P1);
    const uint64_t n2 = pl.passes == 2 && !counted ? hj::scan_state_words(w.tiles2_ub * pl.P2) : 0;
    const uint64_t nw = hj::scan_state_words(w.items_ub * hj::kJoinWaves);
    const uint64_t np = hj::plan_state_words(pl.P);
    static_assert(sizeof(hj::HotKeys) % sizeof(uint64_t) == 0, "hot keys in whole words");
    const uint64_t nq = sizeof(hj::HeavyQueue) / sizeof(uint64_t) + sizeof(hj::HotKeys) / sizeof(uint64_t);
    const uint64_t nc = counted ? 2ull * pl.P : 0;  // totals and cursors: 2 P words of 32 bits each
    uint64_t* zero = c.take<uint64_t>(nq + nc + n1 + n2 + nw + np);
    w.heavy = reinterpret_cast<hj::HeavyQueue*>(zero);
    w.hot = zero ? reinterpret_cast<hj::HotKeys*>(zero + sizeof(hj::HeavyQueue) / sizeof(uint64_t)) : nullptr;
    if (zero) {  // (sizing only when there is no base: no arithmetic on a null pointer)
        if (counted) {
            w.tot2 = reinterpret_cast<uint32_t*>(zero + nq);
            w.cur2 = w.tot2 + 2ull * pl.P;
        }
        w.st1 = zero + nq + nc;
        w.st2 = w.st1 + n1;
        w.stw = w.st2 + n2;
        w.stp = w.stw + nw;
    }
    w.zero = zero;
    w.nzero = nq + nc + n1 + n2 + nw + np;
    w.bytes = c.off;
    return w;
}

// SHJ: the table over R (slots and row chains), then the probe's per-wave counts.
struct ShjTableWs {
    uint64_t* err;
    uint64_t* table;
    uint32_t* next;
    hj::HotKeys* hot;
    uint64_t nslots;
    size_t bytes;
};

ShjTableWs shj_table_layout(uint64_t n_r, void* base) {
    ShjTableWs w{};
    Carver c(base);
    w.nslots = hj::shj_slots(n_r);
    w.err = c.take<uint64_t>(1);
    w.table = c.take<uint64_t>(w.nslots);
    w.next = c.take<uint32_t>(n_r);
    w.hot = c.take<hj::HotKeys>(1);
    w.bytes = c.off;
    return w;
}

struct ShjProbeWs {
    uint64_t* err;
    hj::HeavyQueue* heavy;  // one-pass: heavy S tuples shared by all workgroups
    uint64_t* wave_cnt;
    uint64_t* st;  // scan state of the per-wave counts
    uint64_t nst;
    uint64_t tiles;
    size_t bytes;
};

ShjProbeWs shj_probe_layout(uint64_t n_s, void* base) {
    ShjProbeWs w{};
    Carver c(base);
    w.tiles = cdiv(n_s, hj::kShjTile);
    w.err = c.take<uint64_t>(1);
    w.heavy = c.take<hj::HeavyQueue>(1);
    w.wave_cnt = c.take<uint64_t>(w.tiles * hj::kShjWavesPerBlock);
    w.nst = hj::scan_state_words(w.tiles * hj::kShjWavesPerBlock);
    w.st = c.take<uint64_t>(w.nst);
    w.bytes = c.off;
    return w;
}

size_t shj_bytes(uint64_t n_r, uint64_t n_s) {
    return shj_table_layout(n_r, nullptr).bytes + shj_probe_layout(n_s, nullptr).bytes;
}

// Direct join (PHJ with no partitioning pass): one job descriptor and the item map.
struct DirectWs {
    uint64_t* err;
    hj::DirectJob* job;
    uint32_t* item_job;
    uint32_t nitems;
    size_t bytes;
};

DirectWs direct_layout(uint64_t n_s, void* base) {
    DirectWs w{};
    Carver c(base);
    w.nitems = (uint32_t)cdiv(n_s, hj::kJoinChunk);
    w.err = c.take<uint64_t>(1);
    w.job = c.take<hj::DirectJob>(1);
    w.item_job = c.take<uint32_t>(w.nitems);
    w.bytes = c.off;
    return w;
}

size_t ws_bytes_for(const Plan& pl, uint64_t n_r, uint64_t n_s) {
    if (pl.phj && pl.passes == 0) return direct_layout(n_s, nullptr).bytes;
    return pl.phj ? phj_layout(pl, n_r, n_s, n_r, nullptr).bytes : shj_bytes(n_r, n_s);
}

size_t table_bytes_for(const Plan& pl, uint64_t n_r) {
    if (pl.phj && pl.passes == 0) return kAlign;  // the table is R itself (nothing is stored)
    return pl.phj ? phj_layout(pl, n_r, 0, 0, nullptr).bytes : shj_table_layout(n_r, nullptr).bytes;
}

size_t probe_bytes_for(const Plan& pl, uint64_t n_r, uint64_t n_s) {
    if (pl.phj && pl.passes == 0) return direct_layout(n_s, nullptr).bytes;
    return pl.phj ? phj_layout(pl, 0, n_s, n_r, nullptr).bytes : shj_probe_layout(n_s, nullptr).bytes;
}

void run_direct(const Plan& pl, const hj_rel& R, const hj_rel& S, const hj_out& out, void* ws,
                uint64_t* d_count, hj::Recorder& rec) {
    DirectWs w = direct_layout(S.n, ws);
    hj::DirectJob j{};
    j.rk = R.key;
    j.rr = R.rid;
    j.sk = S.key;
    j.sr = S.rid;
    j.out_r = out.rid_r;
    j.out_s = out.rid_s;
    j.capacity = out.capacity;
    j.count = d_count;
    j.n_r = (uint32_t)R.n;
    j.n_s = (uint32_t)S.n;
    j.item0 = 0;
    hj::direct_setup_one(w.job, w.item_job, j, w.nitems, rec);
    hj::direct_join(w.job, w.item_job, w.nitems, pl.lds_cap, rec);
}

hj_status check_call(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out, void* ws,
                     size_t ws_bytes, uint64_t* d_count, Plan* pl) {
    if (!R || !S || !out) return fail(HJ_ERR_INVALID, "R, S and out must not be NULL");
    hj_status st = check_params(p, R->n, S->n, pl);
    if (st != HJ_OK) return st;
    if (R->n > kMaxRows || S->n > kMaxRows)
        return fail(HJ_ERR_INVALID, "relations must have fewer than 2^31 tuples");
    if (R->n && (!R->key || !R->rid)) return fail(HJ_ERR_INVALID, "R has tuples but a NULL array");
    if (S->n && (!S->key || !S->rid)) return fail(HJ_ERR_INVALID, "S has tuples but a NULL array");
    if (out->capacity && (!out->rid_r || !out->rid_s))
        return fail(HJ_ERR_INVALID, "out has capacity but a NULL array");
    if (!d_count) return fail(HJ_ERR_INVALID, "d_count is NULL");
    const size_t need = ws_bytes_for(*pl, R->n, S->n);
    if (!ws || ws_bytes < need)
        return fail(HJ_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : 0);
    if ((uintptr_t)ws % kAlign) return fail(HJ_ERR_INVALID, "workspace must be 256-byte aligned");
    return HJ_OK;
}

// SHJ build (Algorithm 1, b1-b4): empty slots, then R inserted.
void shj_build_table(const hj_rel& R, const ShjTableWs& t, hj::Recorder& rec) {
    hj::shj_fill(t.table, t.nslots, t.hot, rec);
    hj::shj_build(R.key, R.n, t.table, t.next, t.nslots, t.hot, R.n >= hj::kNtMinBuild, rec);
}

// SHJ probe (Algorithm 1, p1-p4) of a table built over R.
void shj_probe_table(const Plan& pl, const ShjTableWs& t, const hj_rel& R, const hj_rel& S,
                     const hj_out& out, const ShjProbeWs& w, uint64_t* d_count, hj::Recorder& rec) {
    if (!pl.one_pass) {
        hj::shj_count(S.key, S.n, t.table, t.next, t.nslots, R.key, R.n, t.hot, w.wave_cnt, rec);
        hj::zero_words(w.st, w.nst, rec);
        hj::scan_u64(w.wave_cnt, w.wave_cnt, w.tiles * hj::kShjWavesPerBlock, w.st, d_count, rec);
    } else {
        hj::shj_zero_one_pass(d_count, w.heavy, rec);
    }
    hj::shj_write(S.key, S.rid, S.n, t.table, t.next, t.nslots, R.key, R.rid, R.n, t.hot,
                  pl.one_pass ? nullptr : w.wave_cnt, d_count, pl.one_pass ? w.heavy : nullptr, out.rid_r,
                  out.rid_s, out.capacity, rec);
}

void run_shj(const Plan& pl, const hj_rel& R, const hj_rel& S, const hj_out& out, void* ws,
             uint64_t* d_count, hj::Recorder& rec) {
    const ShjTableWs t = shj_table_layout(R.n, ws);
    const ShjProbeWs w = shj_probe_layout(S.n, (char*)ws + t.bytes);
    shj_build_table(R, t, rec);
    shj_probe_table(pl, t, R, S, out, w, d_count, rec);
}

// PHJ partitioning (Algorithm 2, n1-n3) of R and S (either may be empty) into
// w, with the join plan of the partition pairs riding on the last scatter.
// r_pairs: R's partition ranges from a built table (R is then empty here).
// The partitioned arrays are returned in *fk / *fr (R first, S from n_r on).
// *tables_cleared (optional): set when the last scatter cleared the join's HBM tables.
void phj_partition(const Plan& pl, const hj_rel& R, const hj_rel& S, const PhjWs& w, const hj::PartPair* r_pairs,
                   uint64_t* zero_total, int32_t** fk, int32_t** fr, hj::Recorder& rec,
                   bool* tables_cleared = nullptr) {
    if (tables_cleared) *tables_cleared = false;
    const uint32_t n_r = (uint32_t)R.n, n_s = (uint32_t)S.n;
    const bool two = pl.passes == 2;
    const bool counted = two && w.rows;  // (w.rows is set exactly for a counted pass 2 with a workspace)
    hj::Pass1 p1 = hj::make_pass1(R.key, R.rid, n_r, S.key, S.rid, n_s, pl.tile, pl.b1, w.segs1, w.tb1,
                                  w.zero, w.nzero, rec.err_clear);
    if (counted) {
        p1.rows = w.rows;
        p1.esc = w.esc;
        p1.bits_all = pl.B;
    }
    // the join plan rides on the last pass's scatter, the pass-2 setup on the first
    // The plan's records are written at offsets from its chained scan; its wait
    // keeps the full bound and no injected stall (every consumer of the other
    // scans clamps what it reads and writes, the item records have no clamp).
    const hj::ScanCtl plan_ctl{rec.ctl.err, hj::kMaxStatusPolls, 0};
    hj::SideJob plan{};
    plan.kind = hj::kSidePlan;
    plan.blocks = hj::plan_blocks(pl.P, hj::part_block(pl.tile));
    plan.plan = hj::PlanArgs{two ? w.segs2 : w.segs1, two ? w.tb2 : w.tb1, two ? w.hist2 : w.hist1,
                             two ? 2 * pl.P1 : 2u, two ? pl.b2 : pl.b1, n_r, n_s, pl.B, pl.lds_cap,
                             w.pairs, w.item_begin, w.ovf_begin, w.item_rec, w.ovf_part, zero_total, w.stp,
                             r_pairs, plan_ctl, counted ? w.tot2 : nullptr, (uint32_t)w.items_ub};
    hj::SideJob setup2{};
    if (two) {
        setup2.kind = hj::kSideSetup2;
        setup2.blocks = 1;
        setup2.setup2 = hj::Setup2Args{w.hist1, w.tb1, pl.b1, n_r, n_s, pl.tile, pl.b2, 0u, w.keyA, w.ridA,
                                       w.segs2, w.tb2, w.tseg2};
    }
    hj::PassCfg c1{pl.b2, pl.b1, pl.hash, pl.tile, pl.nt_part};
    if (counted) {  // the count rows are summed beside the pass-1 scatter's tiles
        setup2.sums = hj::make_count_sums(w.rows, w.esc, w.tot2, p1.nt_r, p1.ntiles - p1.nt_r, pl.B,
                                          hj::part_block(pl.tile));
        setup2.front = hj::count_sum_blocks(setup2.sums, hj::part_block(pl.tile));
    }
    hj::part_hist_pass1(p1, c1, w.hist1, rec);  // also writes segs1/tb1 and clears the scan states
    hj::scan_u32(w.hist1, w.hist1, w.tiles1 * pl.P1, w.st1, nullptr, rec);
    hj::part_scatter(w.segs1, w.tb1, nullptr, 2, (uint32_t)w.tiles1, c1, w.hist1, w.keyA, w.ridA,
                     two ? setup2 : plan, rec);
    *fk = w.keyA;
    *fr = w.ridA;
    if (two) {
        hj::PassCfg c2{0, pl.b2, pl.hash, pl.tile, pl.nt_part};
        if (counted) {
            // with R scattered here (not a probe of a built table), its HBM tables are cleared by the scatter
            const bool clears = tables_cleared && !r_pairs && hj::counted_clears_tables(pl.b2);
            const hj::Reserve rsv{w.tot2, w.cur2, clears ? w.ovf_table : nullptr, pl.lds_cap, 0u};
            hj::part_scatter(w.segs2, w.tb2, w.tseg2, 2 * pl.P1, (uint32_t)w.tiles2_ub, c2, nullptr, w.keyB,
                             w.ridB, plan, rec, &rsv);
            if (clears) *tables_cleared = true;
        } else {
            hj::part_hist(w.segs2, w.tb2, w.tseg2, 2 * pl.P1, (uint32_t)w.tiles2_ub, c2, w.hist2, rec);
            hj::scan_u32(w.hist2, w.hist2, w.tiles2_ub * pl.P2, w.st2, nullptr, rec);
            hj::part_scatter(w.segs2, w.tb2, w.tseg2, 2 * pl.P1, (uint32_t)w.tiles2_ub, c2, w.hist2, w.keyB,
                             w.ridB, plan, rec);
        }
        *fk = w.keyB;
        *fr = w.ridB;
    }
}

// PHJ join of the planned partition pairs (Algorithm 1 per pair): HBM tables
// for oversized R partitions, then count -> scan -> write (or one-pass write).
// rk/rr: partitioned R, sk/sr: partitioned S.
void phj_join_pairs(const Plan& pl, const PhjWs& w, const int32_t* rk, const int32_t* rr, const int32_t* sk,
                    const int32_t* sr, const hj_out& out, uint64_t* d_count, hj::Recorder& rec,
                    bool tables_cleared = false) {
    hj::join_ovf_build(w.pairs, w.ovf_begin, w.ovf_part, pl.P, (uint32_t)w.ovf_ub, rk, w.ovf_table, w.ovf_next,
                       w.hot, pl.one_pass ? w.heavy : nullptr, rec, !tables_cleared);
    if (!pl.one_pass) {
        hj::join_count(w.pairs, w.item_begin, w.item_rec, pl.P, (uint32_t)w.items_ub, rk, sk, pl.lds_cap,
                       w.ovf_table, w.ovf_next, w.hot, w.wave_cnt, pl.nt_s, rec);
        hj::scan_u64(w.wave_cnt, w.wave_cnt, w.items_ub * hj::kJoinWaves, w.stw, d_count, rec);
    }
    hj::join_write(w.pairs, w.item_begin, w.item_rec, pl.P, (uint32_t)w.items_ub, rk, rr, sk, sr, pl.lds_cap,
                   w.ovf_table, w.ovf_next, pl.one_pass ? nullptr : w.wave_cnt, d_count, out.rid_r, out.rid_s,
                   w.hot, out.capacity, pl.one_pass ? w.heavy : nullptr, pl.nt_s, rec);
}

void run_phj(const Plan& pl, const hj_rel& R, const hj_rel& S, const hj_out& out, void* ws,
             uint64_t* d_count, hj::Recorder& rec) {
    const PhjWs w = phj_layout(pl, R.n, S.n, R.n, ws);
    int32_t *fk, *fr;
    bool cleared = false;
    phj_partition(pl, R, S, w, nullptr, pl.one_pass ? d_count : nullptr, &fk, &fr, rec, &cleared);
    phj_join_pairs(pl, w, fk, fr, fk + R.n, fr + R.n, out, d_count, rec, cleared);
}

void run_join(const Plan& pl, const hj_rel& R, const hj_rel& S, const hj_out& out, void* ws,
              uint64_t* d_count, Recorder& rec) {
    if (R.n == 0 || S.n == 0) {
        hj::write_zero_count(d_count, rec);
    } else if (pl.phj && pl.passes == 0) {
        run_direct(pl, R, S, out, ws, d_count, rec);
    } else if (pl.phj) {
        run_phj(pl, R, S, out, ws, d_count, rec);
    } else {
        run_shj(pl, R, S, out, ws, d_count, rec);
    }
}

void run_build(const Plan& pl, const hj_rel& R, void* ws, hj::Recorder& rec) {
    if (R.n == 0 || (pl.phj && pl.passes == 0)) {  // passes 0: the table is R itself
        hj::zero_pair(rec.err_clear, nullptr, rec);
        return;
    }
    if (!pl.phj) {
        shj_build_table(R, shj_table_layout(R.n, ws), rec);
        return;
    }
    const PhjWs w = phj_layout(pl, R.n, 0, 0, ws);
    const hj_rel none{nullptr, nullptr, 0};
    int32_t *fk, *fr;
    phj_partition(pl, R, none, w, nullptr, nullptr, &fk, &fr, rec);
}

void run_probe(const Plan& pl, const hj_table& t, const hj_rel& S, const hj_out& out, void* ws,
               uint64_t* d_count, hj::Recorder& rec) {
    const hj_rel R{t.r_key, t.r_rid, t.n_r};
    if (t.n_r == 0 || S.n == 0) {
        hj::write_zero_count(d_count, rec);
    } else if (pl.phj && pl.passes == 0) {
        run_direct(pl, R, S, out, ws, d_count, rec);
    } else if (!pl.phj) {
        const ShjTableWs tw = shj_table_layout(t.n_r, t.ws);
        const ShjProbeWs w = shj_probe_layout(S.n, ws);
        shj_probe_table(pl, tw, R, S, out, w, d_count, rec);
    } else {
        // R's partitions and pair ranges are in the table; only S is partitioned here
        const PhjWs tw = phj_layout(pl, t.n_r, 0, 0, t.ws);
        const PhjWs w = phj_layout(pl, 0, S.n, t.n_r, ws);
        const hj_rel none{nullptr, nullptr, 0};
        int32_t *fk, *fr;
        phj_partition(pl, none, S, w, tw.pairs, pl.one_pass ? d_count : nullptr, &fk, &fr, rec);
        const bool two = pl.passes == 2;
        phj_join_pairs(pl, w, two ? tw.keyB : tw.keyA, two ? tw.ridB : tw.ridA, fk, fr, out, d_count, rec);
    }
}

// The plan a table was built with, after checking the table's own fields.
hj_status table_plan(const hj_table* t, uint64_t n_s, Plan* pl) {
    if (!t) return fail(HJ_ERR_INVALID, "table is NULL");
    if (t->n_r > kMaxRows) return fail(HJ_ERR_INVALID, "table: relations must have fewer than 2^31 tuples");
    hj_status st = check_params(&t->params, t->n_r, n_s, pl);
    if (st != HJ_OK) return st;
    if (t->params.algo == HJ_AUTO || (pl->phj && t->params.tile == 0))
        return fail(HJ_ERR_INVALID, "table parameters are not the ones hj_build filled in");
    if (!t->ws || t->ws_bytes < table_bytes_for(*pl, t->n_r))
        return fail(HJ_ERR_INVALID, "table: build workspace missing or too small");
    // SHJ probes read R's rids for every match and scan R's keys for the S
    // tuples of duplicate-heavy keys; PHJ probes without partitioning read both
    const bool reads_r = !pl->phj || pl->passes == 0;
    if (t->n_r && reads_r && (!t->r_rid || !t->r_key))
        return fail(HJ_ERR_INVALID, "table: R's key and rid arrays are needed by this probe");
    return HJ_OK;
}

void init_recorder(Recorder& rec, hipStream_t stream, uint64_t* err, bool clear) {
    rec.stream = stream;
    rec.ctl.err = err;
    rec.err_clear = clear ? err : nullptr;
    rec.ctl.max_polls = kMaxStatusPolls;
    rec.ctl.stall = 0;
    rec.fail_phase = nullptr;
    // HJ_DEBUG_FAIL_PHASE (tests of the failure paths, read per call):
    //   scan_stall     the first tile of every chained scan never publishes and
    //                  waits give up after 64 polls (every kernel still ends;
    //                  the call's error word reports it)
    //   launch:<name>  the launch of phase <name> reports a launch failure
    thread_local std::string phase;
    const char* v = getenv("HJ_DEBUG_FAIL_PHASE");
    if (!v || !*v) return;
    phase = v;
    if (phase == "scan_stall") {
        rec.ctl.max_polls = 64;
        rec.ctl.stall = 1;
    } else if (phase.rfind("launch:", 0) == 0) {
        rec.fail_phase = phase.c_str() + 7;
    }
}

hj_status launch_join(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out, void* ws,
                      size_t ws_bytes, uint64_t* d_count, hj::Recorder& rec) {
    Plan pl;
    hj_status st = check_call(p, R, S, out, ws, ws_bytes, d_count, &pl);
    if (st != HJ_OK) return st;
    (void)hipGetLastError();  // clear a stale error left by unrelated work
    run_join(pl, *R, *S, *out, ws, d_count, rec);
    if (rec.err != hipSuccess)
        return fail(HJ_ERR_DEVICE, "launch failed: %s", hipGetErrorString(rec.err));
    g_err.clear();
    return HJ_OK;
}


}  // namespace eng
}  // namespace hj
