// C ABI (include/hj.h): argument validation, workspace layout and the launch
// sequences of the simple (SHJ) and radix-partitioned (PHJ) hash joins.
//
// SHJ (Algorithm 1): fill table -> build -> count -> scan -> write.
// PHJ (Algorithm 2): per pass: hist -> scan -> scatter (R and S in the same
// launches); then plan the partition pairs -> HBM tables for oversized R
// partitions -> count -> scan -> write.
// Everything is enqueued on the caller's stream; no host synchronisation, no
// host<->device copy and no allocation happen inside hj_join.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hj.h"
#include "hj_internal.h"

namespace {

thread_local std::string g_err;

hj_status fail(hj_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
hj_status fail(hj_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

constexpr size_t kAlign = 256;
constexpr uint64_t kMaxRows = 0x7FFFFFFFull;  // n < 2^31

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

struct Plan {
    bool phj, one_pass;
    uint32_t passes, b1, b2, B, P1, P2, P, tile, hash, lds_cap;
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
// that keeps the same number of write-kernel workgroups per CU.
uint32_t auto_lds_cap(uint64_t n_r, uint32_t P) {
    const double avg = std::ceil((double)n_r / (double)P);
    const double need = avg + 3.0 * std::sqrt(avg) + 32.0;
    uint32_t cap = (uint32_t)std::min<double>(hj::kMaxLdsCap, std::max(256.0, need));
    cap = (cap + 63) / 64 * 64;
    if (cap > hj::kMaxLdsCap) cap = hj::kMaxLdsCap;
    const uint32_t bpc = join_blocks_per_cu(cap);
    while (cap + 64 <= hj::kMaxLdsCap && join_blocks_per_cu(cap + 64) == bpc) cap += 64;
    return cap;
}

hj_status check_params(const hj_params* p, uint64_t n_r, Plan* pl) {
    if (!p) return fail(HJ_ERR_INVALID, "params is NULL");
    if (p->flags & ~HJ_FLAG_ONE_PASS) return fail(HJ_ERR_INVALID, "unknown flags 0x%x", p->flags);
    if (p->algo != HJ_SHJ && p->algo != HJ_PHJ) return fail(HJ_ERR_INVALID, "unknown algo %u", p->algo);
    if (p->hash != HJ_HASH_IDENTITY && p->hash != HJ_HASH_MURMUR2)
        return fail(HJ_ERR_INVALID, "unknown hash %u", p->hash);
    const uint32_t tile = p->tile ? p->tile : 4096;
    if (tile != 1024 && tile != 2048 && tile != 4096 && tile != 8192)
        return fail(HJ_ERR_INVALID, "tile must be 0 or a power of two in 1024..8192 (got %u)", p->tile);
    pl->phj = p->algo == HJ_PHJ;
    pl->one_pass = (p->flags & HJ_FLAG_ONE_PASS) != 0;
    pl->tile = tile;
    pl->hash = p->hash;
    pl->passes = 0;
    pl->b1 = pl->b2 = pl->B = 0;
    pl->P1 = pl->P2 = pl->P = 1;
    pl->lds_cap = 0;
    if (!pl->phj) return HJ_OK;
    if (p->passes != 1 && p->passes != 2) return fail(HJ_ERR_INVALID, "passes must be 1 or 2 (got %u)", p->passes);
    pl->passes = p->passes;
    pl->b1 = p->bits[0];
    pl->b2 = p->passes == 2 ? p->bits[1] : 0;
    if (pl->b1 < 1 || pl->b1 > 13) return fail(HJ_ERR_INVALID, "bits[0] must be in 1..13 (got %u)", pl->b1);
    if (p->passes == 2 && (pl->b2 < 1 || pl->b2 > 13))
        return fail(HJ_ERR_INVALID, "bits[1] must be in 1..13 (got %u)", pl->b2);
    pl->B = pl->b1 + pl->b2;
    if (pl->B > 16) return fail(HJ_ERR_INVALID, "total radix bits must be <= 16 (got %u)", pl->B);
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
    return HJ_OK;
}

// Workspace layout; with base == nullptr only the size is computed.
struct PhjWs {
    hj::PartSeg* segs1;
    uint32_t* tb1;
    uint32_t* hist1;
    int32_t *keyA, *ridA;
    hj::PartSeg* segs2;
    uint32_t* tb2;
    uint32_t* tseg2;
    uint32_t* hist2;
    int32_t *keyB, *ridB;
    hj::PartPair* pairs;
    uint32_t* item_begin;
    uint32_t* ovf_begin;
    uint32_t* item_part;
    uint32_t* ovf_part;
    uint64_t* wave_cnt;
    uint64_t* ovf_table;
    uint32_t* ovf_next;
    uint32_t* part32;
    uint64_t* part64;
    uint64_t tiles1, tiles2_ub, items_ub, ovf_ub;
    size_t bytes;
};

PhjWs phj_layout(const Plan& pl, uint64_t n_r, uint64_t n_s, void* base) {
    PhjWs w{};
    Carver c(base);
    const uint64_t n = n_r + n_s;
    w.tiles1 = cdiv(n_r, pl.tile) + cdiv(n_s, pl.tile);
    w.segs1 = c.take<hj::PartSeg>(2);
    w.tb1 = c.take<uint32_t>(3);
    w.hist1 = c.take<uint32_t>(w.tiles1 * pl.P1);
    w.keyA = c.take<int32_t>(n);
    w.ridA = c.take<int32_t>(n);
    uint64_t hist_max = w.tiles1 * pl.P1;
    if (pl.passes == 2) {
        w.tiles2_ub = cdiv(n, pl.tile) + 2ull * pl.P1;
        w.segs2 = c.take<hj::PartSeg>(2ull * pl.P1);
        w.tb2 = c.take<uint32_t>(2ull * pl.P1 + 1);
        w.tseg2 = c.take<uint32_t>(w.tiles2_ub);
        w.hist2 = c.take<uint32_t>(w.tiles2_ub * pl.P2);
        w.keyB = c.take<int32_t>(n);
        w.ridB = c.take<int32_t>(n);
        hist_max = std::max<uint64_t>(hist_max, w.tiles2_ub * pl.P2);
    }
    w.pairs = c.take<hj::PartPair>(pl.P);
    w.item_begin = c.take<uint32_t>(pl.P + 1ull);
    w.ovf_begin = c.take<uint32_t>(pl.P + 1ull);
    w.items_ub = hj::join_grid(pl.P, n_s);
    w.ovf_ub = hj::ovf_grid(pl.P, n_r);
    w.item_part = c.take<uint32_t>(w.items_ub);
    w.ovf_part = c.take<uint32_t>(w.ovf_ub);
    w.wave_cnt = c.take<uint64_t>(w.items_ub * hj::kJoinWaves);
    w.ovf_table = c.take<uint64_t>(2 * n_r);
    w.ovf_next = c.take<uint32_t>(n_r);
    w.part32 = c.take<uint32_t>(hj::scan_partials(hist_max));
    w.part64 = c.take<uint64_t>(hj::scan_partials(w.items_ub * hj::kJoinWaves));
    w.bytes = c.off;
    return w;
}

struct ShjWs {
    uint64_t* table;
    uint32_t* next;
    uint64_t* wave_cnt;
    uint64_t* part64;
    uint32_t log2_slots;
    uint64_t tiles;
    size_t bytes;
};

ShjWs shj_layout(uint64_t n_r, uint64_t n_s, void* base) {
    ShjWs w{};
    Carver c(base);
    w.log2_slots = std::max<uint32_t>(1, ceil_log2(2 * std::max<uint64_t>(n_r, 1)));
    w.table = c.take<uint64_t>(1ull << w.log2_slots);
    w.next = c.take<uint32_t>(n_r);
    w.tiles = cdiv(n_s, hj::kShjTile);
    w.wave_cnt = c.take<uint64_t>(w.tiles * hj::kShjWavesPerBlock);
    w.part64 = c.take<uint64_t>(hj::scan_partials(w.tiles * hj::kShjWavesPerBlock));
    w.bytes = c.off;
    return w;
}

size_t ws_bytes_for(const Plan& pl, uint64_t n_r, uint64_t n_s) {
    return pl.phj ? phj_layout(pl, n_r, n_s, nullptr).bytes : shj_layout(n_r, n_s, nullptr).bytes;
}

hj_status check_call(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out, void* ws,
                     size_t ws_bytes, uint64_t* d_count, Plan* pl) {
    if (!R || !S || !out) return fail(HJ_ERR_INVALID, "R, S and out must not be NULL");
    hj_status st = check_params(p, R->n, pl);
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

void run_shj(const Plan& pl, const hj_rel& R, const hj_rel& S, const hj_out& out, void* ws,
             uint64_t* d_count, hj::Recorder& rec) {
    ShjWs w = shj_layout(R.n, S.n, ws);
    hj::shj_fill(w.table, 1ull << w.log2_slots, pl.one_pass ? d_count : nullptr, rec);
    hj::shj_build(R.key, R.n, w.table, w.next, w.log2_slots, rec);
    if (!pl.one_pass) {
        hj::shj_count(S.key, S.n, w.table, w.next, w.log2_slots, w.wave_cnt, rec);
        hj::scan_u64(w.wave_cnt, w.wave_cnt, w.tiles * hj::kShjWavesPerBlock, w.part64, d_count, rec);
    }
    hj::shj_write(S.key, S.rid, S.n, w.table, w.next, w.log2_slots, R.rid, pl.one_pass ? nullptr : w.wave_cnt,
                  d_count, out.rid_r, out.rid_s, out.capacity, rec);
}

void run_phj(const Plan& pl, const hj_rel& R, const hj_rel& S, const hj_out& out, void* ws,
             uint64_t* d_count, hj::Recorder& rec) {
    PhjWs w = phj_layout(pl, R.n, S.n, ws);
    const uint32_t n_r = (uint32_t)R.n, n_s = (uint32_t)S.n;
    hj::part_setup_pass1(w.segs1, w.tb1, R.key, R.rid, n_r, S.key, S.rid, n_s, pl.tile, pl.b1, rec);
    hj::PassCfg c1{pl.b2, pl.b1, pl.hash, pl.tile};
    hj::part_hist(w.segs1, w.tb1, nullptr, 2, (uint32_t)w.tiles1, c1, w.hist1, rec);
    hj::scan_u32(w.hist1, w.hist1, w.tiles1 * pl.P1, w.part32, nullptr, rec);
    hj::part_scatter(w.segs1, w.tb1, nullptr, 2, (uint32_t)w.tiles1, c1, w.hist1, w.keyA, w.ridA, rec);
    const hj::PartSeg* segs = w.segs1;
    const uint32_t* tb = w.tb1;
    uint32_t nseg = 2, bits_last = pl.b1;
    const uint32_t* hist_last = w.hist1;
    int32_t *fk = w.keyA, *fr = w.ridA;
    if (pl.passes == 2) {
        hj::part_setup_pass2(w.hist1, w.tb1, pl.b1, n_r, n_s, w.keyA, w.ridA, pl.tile, pl.b2, w.segs2,
                             w.tb2, w.tseg2, rec);
        hj::PassCfg c2{0, pl.b2, pl.hash, pl.tile};
        hj::part_hist(w.segs2, w.tb2, w.tseg2, 2 * pl.P1, (uint32_t)w.tiles2_ub, c2, w.hist2, rec);
        hj::scan_u32(w.hist2, w.hist2, w.tiles2_ub * pl.P2, w.part32, nullptr, rec);
        hj::part_scatter(w.segs2, w.tb2, w.tseg2, 2 * pl.P1, (uint32_t)w.tiles2_ub, c2, w.hist2, w.keyB,
                         w.ridB, rec);
        segs = w.segs2;
        tb = w.tb2;
        nseg = 2 * pl.P1;
        bits_last = pl.b2;
        hist_last = w.hist2;
        fk = w.keyB;
        fr = w.ridB;
    }
    hj::JoinPlanOut po{w.pairs, w.item_begin, w.ovf_begin, w.item_part, w.ovf_part};
    hj::join_plan(segs, tb, nseg, bits_last, hist_last, n_r, n_s, pl.B, pl.lds_cap, po,
                  pl.one_pass ? d_count : nullptr, rec);
    hj::join_ovf_build(w.pairs, w.ovf_begin, w.ovf_part, pl.P, (uint32_t)w.ovf_ub, fk, w.ovf_table, w.ovf_next,
                       rec);
    if (!pl.one_pass) {
        hj::join_count(w.pairs, w.item_begin, w.item_part, pl.P, (uint32_t)w.items_ub, fk, fk + n_r, pl.lds_cap,
                       w.ovf_table, w.ovf_next, w.wave_cnt, rec);
        hj::scan_u64(w.wave_cnt, w.wave_cnt, w.items_ub * hj::kJoinWaves, w.part64, d_count, rec);
    }
    hj::join_write(w.pairs, w.item_begin, w.item_part, pl.P, (uint32_t)w.items_ub, fk, fr, fk + n_r, fr + n_r,
                   pl.lds_cap, w.ovf_table, w.ovf_next, pl.one_pass ? nullptr : w.wave_cnt, d_count,
                   out.rid_r, out.rid_s, out.capacity, rec);
}

hj_status launch_join(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out, void* ws,
                      size_t ws_bytes, uint64_t* d_count, hj::Recorder& rec) {
    Plan pl;
    hj_status st = check_call(p, R, S, out, ws, ws_bytes, d_count, &pl);
    if (st != HJ_OK) return st;
    (void)hipGetLastError();  // clear a stale error left by unrelated work
    if (R->n == 0 || S->n == 0) {
        hj::write_zero_count(d_count, rec);
    } else if (pl.phj) {
        run_phj(pl, *R, *S, *out, ws, d_count, rec);
    } else {
        run_shj(pl, *R, *S, *out, ws, d_count, rec);
    }
    if (rec.err != hipSuccess)
        return fail(HJ_ERR_DEVICE, "launch failed: %s", hipGetErrorString(rec.err));
    g_err.clear();
    return HJ_OK;
}

}  // namespace

namespace hj {

void Recorder::before(const char* name) {
    if (timed && n < cap) {
        names[n] = name;
        hipError_t e = hipEventRecord(ev[2 * n], stream);
        if (e != hipSuccess && err == hipSuccess) err = e;
    }
}

void Recorder::after() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess && err == hipSuccess) err = e;
    if (timed && n < cap) {
        e = hipEventRecord(ev[2 * n + 1], stream);
        if (e != hipSuccess && err == hipSuccess) err = e;
    }
    ++n;
}

}  // namespace hj

extern "C" {

void hj_default_params(hj_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->algo = HJ_PHJ;
    p->passes = 2;
    p->bits[0] = 6;
    p->bits[1] = 6;
    p->hash = HJ_HASH_IDENTITY;
    p->tile = 4096;
    p->lds_cap = 0;
    p->flags = 0;
}

size_t hj_workspace_bytes(const hj_params* p, uint64_t n_r, uint64_t n_s) {
    Plan pl;
    if (check_params(p, n_r, &pl) != HJ_OK) return 0;
    if (n_r > kMaxRows || n_s > kMaxRows) {
        fail(HJ_ERR_INVALID, "relations must have fewer than 2^31 tuples");
        return 0;
    }
    return ws_bytes_for(pl, n_r, n_s);
}

hj_status hj_join(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out, void* ws,
                  size_t ws_bytes, uint64_t* d_count, void* stream) {
    hj::Recorder rec;
    rec.stream = (hipStream_t)stream;
    return launch_join(p, R, S, out, ws, ws_bytes, d_count, rec);
}

hj_status hj_join_sync(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out, void* ws,
                       size_t ws_bytes, uint64_t* d_count, uint64_t* h_count, void* stream) {
    if (!h_count) return fail(HJ_ERR_INVALID, "h_count is NULL");
    hj_status st = hj_join(p, R, S, out, ws, ws_bytes, d_count, stream);
    if (st != HJ_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(h_count, d_count, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(HJ_ERR_DEVICE, "synchronisation failed: %s", hipGetErrorString(e));
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
    rec.stream = (hipStream_t)stream;
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

const char* hj_last_error(void) { return g_err.c_str(); }

uint32_t hj_version(void) { return 100; }

}  // extern "C"
