// Joins of relations held in host memory that are larger than the device can
// hold at once: the paper's joins of datasets beyond its zero-copy buffer
// (appendix "More Experimental Results", "Large datasets that cannot fit into
// the zero copy buffer"), done like a classic external-memory hash join with
// device memory as the main memory and host memory as the external memory.
//
//  1. Partition pass: R, then S, streams through the device in chunks; every
//     chunk is split into 2^k partitions on the k high bits of the key's
//     MurmurHash 2.0 with the radix kernels of Algorithm 2 (histogram, scan,
//     scatter: phj_partition.hip), and the partitioned chunk goes back to a
//     pinned host buffer together with its partition boundaries.  Two device
//     slots on two streams alternate, so one chunk's copies overlap the other
//     chunk's kernels and copies (host->device and device->host run together).
//  2. Link: partition i of R (of S) is the list of partition-i runs of all
//     R (S) chunks; nothing is moved.
//  3. Join: each partition pair is copied to the device run by run and joined
//     by the single-join engine with the caller's parameters (the in-memory
//     PHJ partitions on the key's low bits or on MurmurHash 2.0's low bits,
//     independent of the k high bits used here); its pairs are copied to the
//     host output.  An S partition too large for the device together with its
//     R partition, or whose pairs overflow the device output buffer, is joined
//     in pieces against the whole R partition.
// The k = 0 case (everything fits) skips the partition pass, as in the paper.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/hj.h"
#include "engine.h"
#include "hj_internal.h"
#include "hj_side.h"

using namespace hj::eng;

namespace {

using Clock = std::chrono::steady_clock;

constexpr uint32_t kExtTile = 8192;           // partitioning tile of the chunks
constexpr uint64_t kMaxChunk = 1ull << 28;    // tuples per chunk (and per device slot)
constexpr uint32_t kMaxFanoutBits = 13;       // one radix pass
constexpr size_t kMinExternalWs = 64ull << 20;

struct Carve {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(uint64_t count) {
        T* p = base ? (T*)(base + off) : nullptr;
        off += align_up(sizeof(T) * (size_t)std::max<uint64_t>(count, 1));
        return p;
    }
};

// One device slot of the partition pass: a chunk of up to c tuples, its
// partitioned copy, histogram, scan state and partition boundaries.
struct Slot {
    hj::PartSeg* segs;
    uint32_t* tb;
    uint32_t* hist;
    int32_t *kin, *rin, *kout, *rout;
    uint64_t* st;
    uint64_t nst;
    uint32_t* starts;
    size_t bytes;
};

Slot slot_layout(uint64_t c, uint32_t k, char* base) {
    Slot s{};
    Carve cv{base};
    const uint64_t tiles = cdiv(c, kExtTile);
    s.segs = cv.take<hj::PartSeg>(2);
    s.tb = cv.take<uint32_t>(3);
    s.hist = cv.take<uint32_t>(tiles << k);
    s.kin = cv.take<int32_t>(c);
    s.rin = cv.take<int32_t>(c);
    s.kout = cv.take<int32_t>(c);
    s.rout = cv.take<int32_t>(c);
    s.nst = hj::scan_state_words(tiles << k);
    s.st = cv.take<uint64_t>(s.nst);
    s.starts = cv.take<uint32_t>((1ull << k) + 1);
    s.bytes = cv.off;
    return s;
}

// A run of tuples in host memory: key[0..n), rid[0..n).
struct Run {
    const int32_t* key;
    const int32_t* rid;
    uint64_t n;
};

// Device bytes a pair of r and s tuples needs: inputs, join workspace and room
// for `out` pairs.
size_t pair_bytes(const hj_params* p, uint64_t r, uint64_t s, uint64_t out) {
    Plan pl;
    if (check_params(p, r, s, &pl) != HJ_OK) return ~(size_t)0;
    // error word, four input columns, count, join workspace, two output columns
    return 3 * kAlign + 4 * align_up(4 * std::max<uint64_t>(r, s)) + ws_bytes_for(pl, r, s) + 2 * align_up(4 * out);
}

struct Ctx {
    const hj_params* p;
    char* ws;
    size_t ws_bytes;
    uint64_t* err;
    hipStream_t stream;
    uint64_t* h_cnt;  // pinned
    uint64_t total = 0;
    const hj_out* out;
    uint64_t h2d = 0, d2h = 0;
    uint32_t pieces = 0;
};

hj_status hip_fail(const char* what, hipError_t e) {
    return fail(HJ_ERR_DEVICE, "%s failed: %s", what, hipGetErrorString(e));
}

// Copies tuples [a, b) of the concatenation of `runs` to dk/dr.
hipError_t copy_runs(const std::vector<Run>& runs, uint64_t a, uint64_t b, int32_t* dk, int32_t* dr,
                     hipStream_t s, uint64_t* bytes) {
    uint64_t pos = 0, at = 0;
    for (const Run& r : runs) {
        const uint64_t lo = std::max(a, pos), hi = std::min(b, pos + r.n);
        if (lo < hi) {
            const size_t nb = 4 * (hi - lo);
            hipError_t e = hipMemcpyAsync(dk + at, r.key + (lo - pos), nb, hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync(dr + at, r.rid + (lo - pos), nb, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return e;
            at += hi - lo;
            *bytes += 2 * nb;
        }
        pos += r.n;
        if (pos >= b) break;
    }
    return hipSuccess;
}

// Joins the pair (R runs, S runs) on the device, S in pieces when needed.
hj_status join_pair(Ctx& C, const std::vector<Run>& rr, uint64_t nr, const std::vector<Run>& sr, uint64_t ns) {
    if (nr == 0 || ns == 0) return HJ_OK;
    // the largest S piece (at most all of S) that fits with R and an output of
    // at least one pair per S tuple
    uint64_t piece = ns;
    while (piece > 0 && pair_bytes(C.p, nr, piece, piece) > C.ws_bytes) piece /= 2;
    if (piece == 0 || pair_bytes(C.p, nr, std::min<uint64_t>(ns, 4096), std::min<uint64_t>(ns, 4096)) > C.ws_bytes)
        return fail(HJ_ERR_WORKSPACE,
                    "a partition of %llu R tuples does not fit the %zu-byte workspace with its join (a key with "
                    "too many duplicates, or too small a workspace)",
                    (unsigned long long)nr, C.ws_bytes);
    uint64_t a = 0;
    while (a < ns) {
        const uint64_t b = std::min(ns, a + piece);
        const uint64_t sn = b - a;
        Plan pl;
        hj_status st = check_params(C.p, nr, sn, &pl);
        if (st != HJ_OK) return st;
        Carve cv{C.ws};
        cv.take<uint64_t>(1);  // the call's error word
        int32_t* rk = cv.take<int32_t>(nr);
        int32_t* rrid = cv.take<int32_t>(nr);
        int32_t* sk = cv.take<int32_t>(sn);
        int32_t* srid = cv.take<int32_t>(sn);
        uint64_t* d_count = cv.take<uint64_t>(1);
        const size_t jws_bytes = ws_bytes_for(pl, nr, sn);
        char* jws = cv.take<char>(jws_bytes);
        const size_t used = cv.off;
        const uint64_t cap = used + 2 * kAlign < C.ws_bytes ? (C.ws_bytes - used - 2 * kAlign) / 8 : 0;
        int32_t* o_r = (int32_t*)(C.ws + used);
        int32_t* o_s = (int32_t*)(C.ws + used + align_up(4 * cap));
        hipError_t e = copy_runs(rr, 0, nr, rk, rrid, C.stream, &C.h2d);
        if (e == hipSuccess) e = copy_runs(sr, a, b, sk, srid, C.stream, &C.h2d);
        if (e != hipSuccess) return hip_fail("host-to-device copy", e);
        const hj_rel R{rk, rrid, nr}, S{sk, srid, sn};
        const hj_out O{o_r, o_s, cap};
        hj::Recorder rec;
        init_recorder(rec, C.stream, C.err, false);
        st = launch_join(C.p, &R, &S, &O, jws, jws_bytes, d_count, rec);
        if (st != HJ_OK) return st;
        e = hipMemcpyAsync(C.h_cnt, d_count, sizeof(uint64_t), hipMemcpyDeviceToHost, C.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(C.stream);
        if (e != hipSuccess) return hip_fail("join synchronisation", e);
        ++C.pieces;
        const uint64_t cnt = *C.h_cnt;
        if (cnt > cap) {  // more pairs than the device output holds: smaller S pieces
            if (sn == 1) return fail(HJ_ERR_WORKSPACE, "one S tuple has more pairs than the workspace holds");
            piece = std::max<uint64_t>(1, sn / 2);
            continue;
        }
        // the piece's pairs to the host output, up to its capacity
        const uint64_t keep = C.total < C.out->capacity ? std::min(cnt, C.out->capacity - C.total) : 0;
        if (keep) {
            e = hipMemcpyAsync(C.out->rid_r + C.total, o_r, 4 * keep, hipMemcpyDeviceToHost, C.stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(C.out->rid_s + C.total, o_s, 4 * keep, hipMemcpyDeviceToHost, C.stream);
            if (e == hipSuccess) e = hipStreamSynchronize(C.stream);
            if (e != hipSuccess) return hip_fail("device-to-host copy", e);
            C.d2h += 8 * keep;
        }
        C.total += cnt;
        a = b;
    }
    return HJ_OK;
}

// Smallest fan-out whose expected largest partition pair fits the workspace.
uint32_t plan_fanout(const hj_params* p, uint64_t n_r, uint64_t n_s, size_t ws_bytes) {
    for (uint32_t k = 0; k <= kMaxFanoutBits; ++k) {
        const double P = std::ldexp(1.0, (int)k);
        auto expect = [&](uint64_t n) {
            const double m = (double)n / P;
            return k == 0 ? (uint64_t)n : (uint64_t)std::ceil(m * 1.02 + 6.0 * std::sqrt(m) + 64.0);
        };
        const uint64_t r = expect(n_r), s = expect(n_s);
        if (pair_bytes(p, r, s, s) <= ws_bytes) return k;
    }
    return kMaxFanoutBits;
}

// Partitions relation X (host arrays) chunk by chunk into the pinned host
// arrays hk/hr at the same positions; records every chunk's partition
// boundaries in `starts` (chunk-major, 2^k + 1 per chunk).
hj_status partition_relation(const hj_rel& X, uint32_t k, uint64_t chunk, Slot* slots, hipStream_t* streams,
                             uint64_t* err, int32_t* hk, int32_t* hr, uint32_t* starts, uint64_t* h2d,
                             uint64_t* d2h) {
    const uint32_t P = 1u << k;
    const uint64_t nchunks = cdiv(X.n, chunk);
    for (uint64_t j = 0; j < nchunks; ++j) {
        Slot& sl = slots[j & 1];
        hipStream_t s = streams[j & 1];
        const uint64_t off = j * chunk;
        const uint32_t len = (uint32_t)std::min<uint64_t>(chunk, X.n - off);
        hipError_t e = hipMemcpyAsync(sl.kin, X.key + off, 4ull * len, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(sl.rin, X.rid + off, 4ull * len, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail("host-to-device copy", e);
        *h2d += 8ull * len;
        hj::Recorder rec;
        init_recorder(rec, s, err, false);
        const hj::Pass1 p1 = hj::make_pass1(sl.kin, sl.rin, len, nullptr, nullptr, 0, kExtTile, k, sl.segs, sl.tb,
                                            sl.st, sl.nst, nullptr);
        const hj::PassCfg cfg{32 - k, k, HJ_HASH_MURMUR2, kExtTile, len >= hj::kNtMinTuples};
        const uint32_t tiles = (uint32_t)cdiv(len, kExtTile);
        hj::part_hist_pass1(p1, cfg, sl.hist, rec);
        hj::scan_u32(sl.hist, sl.hist, (uint64_t)tiles << k, sl.st, nullptr, rec);
        hj::SideJob none{};
        hj::part_scatter(sl.segs, sl.tb, nullptr, 2, tiles, cfg, sl.hist, sl.kout, sl.rout, none, rec);
        hj::part_starts(sl.hist, tiles, k, len, sl.starts, rec);
        if (rec.err != hipSuccess) return hip_fail("partition launch", rec.err);
        e = hipMemcpyAsync(hk + off, sl.kout, 4ull * len, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(hr + off, sl.rout, 4ull * len, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(starts + j * (P + 1ull), sl.starts, 4ull * (P + 1), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return hip_fail("device-to-host copy", e);
        *d2h += 8ull * len;
    }
    return HJ_OK;
}

struct Host {
    int32_t* buf = nullptr;    // pinned: keys of R then S, rids of R then S
    uint32_t* starts = nullptr;  // pinned
    uint64_t* cnt = nullptr;     // pinned
    hipStream_t st[2] = {nullptr, nullptr};
    ~Host() {
        for (hipStream_t s : st)
            if (s) (void)hipStreamDestroy(s);
        if (buf) (void)hipHostFree(buf);
        if (starts) (void)hipHostFree(starts);
        if (cnt) (void)hipHostFree(cnt);
    }
};

}  // namespace

extern "C" {

hj_status hj_join_external(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out, void* ws,
                           size_t ws_bytes, uint64_t* h_count, hj_external_info* info) {
    if (!p || !R || !S || !out || !h_count) return fail(HJ_ERR_INVALID, "p, R, S, out and h_count must be given");
    if (R->n > kMaxRows || S->n > kMaxRows) return fail(HJ_ERR_INVALID, "relations must have fewer than 2^31 tuples");
    if ((R->n && (!R->key || !R->rid)) || (S->n && (!S->key || !S->rid)))
        return fail(HJ_ERR_INVALID, "a relation has tuples but a NULL array");
    if (out->capacity && (!out->rid_r || !out->rid_s)) return fail(HJ_ERR_INVALID, "out has capacity but a NULL array");
    Plan probe_plan;
    hj_status st = check_params(p, R->n, S->n, &probe_plan);
    if (st != HJ_OK) return st;
    if (!ws || ws_bytes < kMinExternalWs)
        return fail(HJ_ERR_WORKSPACE, "hj_join_external needs a workspace of at least %zu bytes", kMinExternalWs);
    if ((uintptr_t)ws % kAlign) return fail(HJ_ERR_INVALID, "workspace must be 256-byte aligned");
    const Clock::time_point t0 = Clock::now();
    hj_external_info inf{};
    *h_count = 0;
    Host H;
    hipError_t e = hipHostMalloc((void**)&H.cnt, sizeof(uint64_t), hipHostMallocDefault);
    for (int i = 0; e == hipSuccess && i < 2; ++i) e = hipStreamCreateWithFlags(&H.st[i], hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail("stream / pinned count setup", e);
    (void)hipGetLastError();
    char* base = (char*)ws;
    uint64_t* err = (uint64_t*)base;
    {
        hj::Recorder rec;
        init_recorder(rec, H.st[0], err, false);
        hj::zero_pair(err, nullptr, rec);
        e = rec.err != hipSuccess ? rec.err : hipStreamSynchronize(H.st[0]);
        if (e != hipSuccess) return hip_fail("workspace setup", e);
    }
    Ctx C{p, base, ws_bytes, err, H.st[0], H.cnt};
    C.out = out;
    const uint32_t k = (R->n && S->n) ? plan_fanout(p, R->n, S->n, ws_bytes) : 0;
    inf.fanout_bits = k;
    if (R->n == 0 || S->n == 0) {
        // no pairs
    } else if (k == 0) {
        // everything fits: one pair, no partition pass
        const std::vector<Run> rr{Run{R->key, R->rid, R->n}}, sr{Run{S->key, S->rid, S->n}};
        const Clock::time_point t1 = Clock::now();
        st = join_pair(C, rr, R->n, sr, S->n);
        inf.join_s = std::chrono::duration<double>(Clock::now() - t1).count();
        if (st != HJ_OK) return st;
    } else {
        const uint32_t P = 1u << k;
        // two device slots for chunks of up to `chunk` tuples
        const size_t avail = ws_bytes - kAlign;
        uint64_t chunk = kMaxChunk;
        while (chunk > kExtTile && 2 * slot_layout(chunk, k, nullptr).bytes > avail) chunk /= 2;
        if (2 * slot_layout(chunk, k, nullptr).bytes > avail)
            return fail(HJ_ERR_WORKSPACE, "workspace too small for the partition pass");
        inf.chunk_tuples = chunk;
        Slot slots[2] = {slot_layout(chunk, k, base + kAlign), slot_layout(chunk, k, nullptr)};
        slots[1] = slot_layout(chunk, k, base + kAlign + align_up(slots[0].bytes));
        const uint64_t N = R->n + S->n;
        const uint64_t cr = cdiv(R->n, chunk), cs = cdiv(S->n, chunk);
        e = hipHostMalloc((void**)&H.buf, 8ull * N, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&H.starts, 4ull * (cr + cs) * (P + 1ull), hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail("pinned host buffer for the partitions", e);
        int32_t* hk = H.buf;
        int32_t* hr = H.buf + N;
        const Clock::time_point t1 = Clock::now();
        st = partition_relation(*R, k, chunk, slots, H.st, err, hk, hr, H.starts, &C.h2d, &C.d2h);
        if (st == HJ_OK)
            st = partition_relation(*S, k, chunk, slots, H.st, err, hk + R->n, hr + R->n, H.starts + cr * (P + 1ull),
                                    &C.h2d, &C.d2h);
        for (int i = 0; i < 2; ++i) {
            e = hipStreamSynchronize(H.st[i]);
            if (e != hipSuccess && st == HJ_OK) st = hip_fail("partition pass", e);
        }
        if (st != HJ_OK) return st;
        const Clock::time_point t2 = Clock::now();
        inf.partition_s = std::chrono::duration<double>(t2 - t1).count();
        // link: partition i = the partition-i runs of every chunk
        std::vector<Run> rr, sr;
        for (uint32_t i = 0; i < P; ++i) {
            rr.clear();
            sr.clear();
            uint64_t nr = 0, ns = 0;
            for (uint64_t j = 0; j < cr + cs; ++j) {
                const uint32_t* b = H.starts + j * (P + 1ull);
                const uint64_t n = b[i + 1] - b[i];
                if (!n) continue;
                const uint64_t at = j * chunk - (j < cr ? 0 : cr * chunk) + (j < cr ? 0 : R->n) + b[i];
                const Run run{hk + at, hr + at, n};
                if (j < cr) {
                    rr.push_back(run);
                    nr += n;
                } else {
                    sr.push_back(run);
                    ns += n;
                }
            }
            st = join_pair(C, rr, nr, sr, ns);
            if (st != HJ_OK) return st;
        }
        inf.join_s = std::chrono::duration<double>(Clock::now() - t2).count();
    }
    uint64_t werr = 0;
    e = hipMemcpy(&werr, err, sizeof(uint64_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail("error word read", e);
    inf.pieces = C.pieces;
    inf.h2d_bytes = C.h2d;
    inf.d2h_bytes = C.d2h;
    inf.total_s = std::chrono::duration<double>(Clock::now() - t0).count();
    if (info) *info = inf;
    *h_count = C.total;
    if (werr) return fail(HJ_ERR_DEVICE, "device error word 0x%llx: a chained scan gave up", (unsigned long long)werr);
    if (C.total > out->capacity)
        return fail(HJ_ERR_CAPACITY, "%llu pairs do not fit capacity %llu", (unsigned long long)C.total,
                    (unsigned long long)out->capacity);
    clear_error();
    return HJ_OK;
}

}  // extern "C"
