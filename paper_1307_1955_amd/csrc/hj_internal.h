// Internal declarations shared by the engine (hj_api.cpp) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace hj {

// One input segment of a partitioning pass.  A pass partitions every segment
// independently: the tuples of segment s land in [out_base, out_base + n) of
// the output arrays, grouped by partition number.
struct PartSeg {
    const int32_t* key_in;
    const int32_t* rid_in;
    uint64_t out_base;   // first output position of this segment
    uint64_t hist_base;  // first histogram entry of this segment (ntiles * P entries)
    uint32_t n;          // tuples
    uint32_t pad;
};

// One join work item: an R partition and a chunk of its S partition
// (positions relative to each relation's base in the scratch arrays).
struct ItemRec {
    uint32_t r_off, r_len;
    uint32_t s_begin, s_n;
};

// One final partition pair of a PHJ: ranges in the partitioned R and S arrays
// (positions relative to each relation's base in the scratch arrays).
struct PartPair {
    uint32_t r_off, r_len;
    uint32_t s_off, s_len;
};

// Bound on the polls of one unset status in a chained scan (decoupled
// look-back): predecessors always publish (they took their tickets earlier and
// wait on nothing later), the bound only guarantees that a kernel ends.
constexpr uint32_t kMaxStatusPolls = 1u << 20;
// Bits of a call's device error word (the first 8 bytes of its workspace; the
// call's first kernel clears it).
constexpr uint64_t kErrLookback = 1;  // a chained scan gave up waiting for a predecessor
// How the chained scans of one call wait, and where a scan that gives up says so.
struct ScanCtl {
    uint64_t* err;       // the call's error word (kErrLookback is or-ed in)
    uint32_t max_polls;  // polls of one unset status before giving up
    uint32_t stall;      // failure injection: the first tile of every chained scan never publishes
};

// Launch recorder: the stream, the call's error word, optional per-launch HIP
// event timing, and the first launch error.
struct Recorder {
    hipStream_t stream = nullptr;
    ScanCtl ctl{nullptr, kMaxStatusPolls, 0};
    // the call's first kernel clears this word (nullptr: the word belongs to an
    // enclosing batch that cleared it already)
    uint64_t* err_clear = nullptr;
    // failure injection: the launch of this phase reports a launch failure
    const char* fail_phase = nullptr;
    const char* cur = nullptr;
    bool timed = false;
    uint32_t n = 0, cap = 0;
    const char** names = nullptr;
    hipEvent_t* ev = nullptr;  // 2 per launch
    hipError_t err = hipSuccess;
    void before(const char* name);
    void after();
};

// ---- scan.hip ----
// Exclusive scans in one launch.  `state` needs scan_state_words(n) words that
// are zero when the scan starts (it leaves them non-zero).  `in` may equal `out`.
size_t scan_state_words(uint64_t n);
void scan_u32(const uint32_t* in, uint32_t* out, uint64_t n, uint64_t* state, uint32_t* total, Recorder& rec);
void scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* state, uint64_t* total, Recorder& rec);
// Clears n words.
void zero_words(uint64_t* p, uint64_t n, Recorder& rec);
// Clears the words a and b (either may be nullptr) in one small launch.
void zero_pair(uint64_t* a, uint64_t* b, Recorder& rec);

// ---- shj.hip ----
constexpr uint32_t kShjBlock = 256;
constexpr uint32_t kShjTile = 2048;  // S tuples per probe tile
constexpr uint32_t kShjWavesPerBlock = kShjBlock / 64;
// Slots of the SHJ table per R row (linear probing, load factor 1 / this).
constexpr double kShjSlotsPerRow = 2.0;
// Slots of the SHJ table over n_r rows: kShjSlotsPerRow per row, rounded up to
// whole 128-byte lines.
inline uint64_t shj_slots(uint64_t n_r) {
    const uint64_t s = (uint64_t)(kShjSlotsPerRow * (double)(n_r < 1 ? 1 : n_r) + 0.999999);
    return (s + 15) / 16 * 16;
}
struct HotKeys;  // keys the build saw in long push runs (hj_device.h)
// Fills the table with empty slots, clears the hot-key record and the call's
// error word (rec.err_clear).
void shj_fill(uint64_t* table, uint64_t nslots, HotKeys* hot, Recorder& rec);
// nt: R's keys read with non-temporal loads (kNtMinBuild).
void shj_build(const int32_t* key, uint64_t n, uint64_t* table, uint32_t* next, uint64_t nslots,
               HotKeys* hot, bool nt, Recorder& rec);
// Heavy S tuples of a one-pass probe (SHJ, and the HBM-table partitions of
// PHJ) are handed to a device-wide queue: any workgroup that has finished its
// own work claims chunks of the tuple's R rows and writes their matches (one
// 64-byte record per tuple; the queue is zeroed before each probe).
constexpr uint32_t kHeavyJobs = 256;
constexpr uint32_t kHelpChunk = 1u << 16;  // R rows per claimed chunk
struct HeavyJob {
    int32_t key, srid;
    uint32_t valid;        // 1 once the fields below are written
    uint32_t write_next;   // next chunk to claim
    uint32_t r_off, r_len; // the R rows that hold the tuple's matches (SHJ: all of R)
    uint32_t pad[10];
};
struct HeavyQueue {
    uint32_t n;            // tuples handed in (may exceed kHeavyJobs: the rest stay with their workgroup)
    // PHJ one-pass write: the HBM-table build sets `wait` when a partition can
    // hand tuples in (more than kHelpChunk rows) and adds that partition's
    // work items to items_expected; those items count themselves done, and the
    // write's helper workgroups help the queue until items_done reaches
    // items_expected
    uint32_t wait;
    uint32_t items_expected;
    uint32_t items_done;
    uint32_t pad[12];
    HeavyJob job[kHeavyJobs];
};
static_assert(sizeof(HeavyJob) == 64 && sizeof(HeavyQueue) % 8 == 0, "queue layout");
// Sets *d_count to zero and empties the queue (one-pass SHJ probes); clears
// the call's error word (rec.err_clear).
void shj_zero_one_pass(uint64_t* d_count, HeavyQueue* q, Recorder& rec);

// The probe kernels read R's columns (r_key, r_rid, n_r rows, the ones the
// table was built from) for keys with long chains.  shj_count also clears the
// call's error word (rec.err_clear): it runs before the count scan.
void shj_count(const int32_t* s_key, uint64_t n_s, const uint64_t* table, const uint32_t* next,
               uint64_t nslots, const int32_t* r_key, uint64_t n_r, const HotKeys* hot, uint64_t* wave_cnt,
               Recorder& rec);
void shj_write(const int32_t* s_key, const int32_t* s_rid, uint64_t n_s, const uint64_t* table,
               const uint32_t* next, uint64_t nslots, const int32_t* r_key, const int32_t* r_rid,
               uint64_t n_r, const HotKeys* hot, const uint64_t* wave_base, uint64_t* total, HeavyQueue* heavy,
               int32_t* out_r, int32_t* out_s, uint64_t capacity,
               Recorder& rec);  // wave_base == nullptr: one-pass output into *total

// ---- phj_partition.hip ----
// Threads of a partitioning workgroup for a given tile: 512 from 4096 tuples on
// (twice the waves per CU of 256-thread workgroups at the same LDS per tile;
// measured on MI355X: the 8192-tuple scatter 1.3x faster, the 16M x 16M join
// 4% faster), 256 below (the vector tile loads need >= 4 tuples per thread).
constexpr uint32_t kMinPartBlock = 256;
inline uint32_t part_block(uint32_t tile) { return tile >= 4096 ? 512u : kMinPartBlock; }
// Default partitioning tile: 8192 tuples when the join has enough tuples to
// fill the chip several times over with such tiles and needs the longer
// partition runs they give (2^25 tuples or more, or 2^24 or more in one pass of
// 8 or more radix bits), else 4096 (measured on MI355X).
inline uint32_t default_tile(uint64_t n_r, uint64_t n_s, uint32_t passes, uint32_t bits1) {
    const uint64_t n = n_r + n_s;
    return (n >= (1ull << 25) || (n >= (1ull << 24) && passes == 1 && bits1 >= 8)) ? 8192u : 4096u;
}
struct PassCfg {
    uint32_t shift;      // radix bits taken from (hash >> shift)
    uint32_t bits;       // partitions = 1 << bits
    uint32_t hash_kind;  // hj_hash
    uint32_t tile;       // tuples per tile
    uint32_t nt;         // tiles read with non-temporal loads
};
// Non-temporal loads of data a launch reads once pay only once a join's
// relations outgrow the caches; below that, plain loads leave lines that a
// later launch reads again.  Measured on MI355X (PHJ, one-pass output):
// partitioning tiles from |R| + |S| = 2^24 on (8M x 16M: -3.7%, 16M x 16M:
// -5.8%; 1M x 4M: +5.7%, 4M x 8M: +1.6%), the join's S chunks only while
// also |S| <= 2 |R| (16M x 16M: -1.2%; 2M x 16M and 16M x 64M: +1.5%), the
// SHJ build's R keys from |R| = 2^23 (16M: -7% build time; the probe's S
// loads gained nothing and stay plain).
constexpr uint64_t kNtMinTuples = 1ull << 24;
constexpr uint64_t kNtMinBuild = 1ull << 23;
// Two passes whose final partitions number 2^4..2^kCountedMaxBits are
// "counted": pass 1 also counts every tile's tuples per final partition (one
// row of 2^bits 8-bit counts per tile; a count of 255 or more is 0 in the row
// and goes to the tile's list of kCountEsc escapes instead: a tile of at most
// 8192 tuples has no more than 32 of them), workgroups at the front of the
// pass-1 scatter sum the rows into per-relation totals, and pass 2 has no
// histogram of its own: each pass-2 tile places its runs at the scanned
// totals of its segment plus what it reserves on a cursor per final
// partition (the order of tiles inside a partition is then the order of
// their reservations).  More bits would make the rows larger than the pass-2
// histogram read they replace.
constexpr uint32_t kCountedMaxBits = 13;
constexpr uint32_t kCountEsc = 32;       // escapes per tile: (partition << 14) | count, 0 unused
constexpr uint32_t kCountEscMin = 255;   // counts from here on are escaped
inline bool counted_pass2(uint32_t passes, uint32_t b1, uint32_t b2) {
    return passes == 2 && b1 + b2 >= 4 && b1 + b2 <= kCountedMaxBits;
}
// A counted pass 2's totals and cursors, each 2^(b1 + b2) entries for R then
// as many for S (index = segment * 2^b2 + partition in the segment).
struct Reserve {
    const uint32_t* tot;
    uint32_t* cur;  // zero before the pass
    // Optional (nullptr: not done here): the HBM tables of R's partitions of more
    // than lds_cap tuples (2 slots per tuple at twice its position in R) are
    // cleared by the tiles that write the partitions' runs, in place of the
    // clearing launch.  Only with at most 64 partitions per segment.
    uint64_t* ovf_table;
    uint32_t lds_cap, pad;
};
// Whether a counted pass 2 clears the HBM tables (Reserve::ovf_table).
inline bool counted_clears_tables(uint32_t b2) { return b2 <= 6; }
// The sums of a counted pass 2's count rows (Pass1::rows and ::esc: nt_r
// rows of R, then nt_s of S) into tot[rel * 2^bits + i] (zero before), by
// workgroups at the front of the pass-1 scatter's grid: the totals are needed
// only by pass 2, so the sums run beside the scatter's tiles.  Each workgroup
// takes `rows_per` rows of one relation and a group of 16-count columns
// (spread over its threads in phases when the group is narrower than it).
struct CountSums {
    const uint8_t* rows;
    const uint32_t* esc;
    uint32_t* tot;
    uint32_t nt_r, nt_s, bits, rows_per;
};
// Column groups of 16-count columns per row for workgroups of `block` threads.
__host__ __device__ inline uint32_t count_sum_groups(uint32_t bits, uint32_t block) {
    const uint32_t cols = (1u << bits) / 16;
    return cols > block ? cols / block : 1u;
}
// About 32 workgroups in all: each adds its sums with atomics, and the pass-1
// scatter they run beside leaves them time for many rows; 8 rows at least.
inline CountSums make_count_sums(const uint8_t* rows, const uint32_t* esc, uint32_t* tot, uint32_t nt_r,
                                 uint32_t nt_s, uint32_t bits, uint32_t block) {
    const uint64_t want = ((uint64_t)(nt_r + nt_s) * count_sum_groups(bits, block) + 31) / 32;
    return CountSums{rows, esc, tot, nt_r, nt_s, bits, want > 8 ? (uint32_t)want : 8u};
}
// Workgroups of the sums, rounded up to a multiple of 8 (the scatter's tiles
// keep their XCD mapping behind them; the extra ones have no rows).
inline uint32_t count_sum_blocks(const CountSums& c, uint32_t block) {
    const uint32_t b = count_sum_groups(c.bits, block) *
                       ((c.nt_r + c.rows_per - 1) / c.rows_per + (c.nt_s + c.rows_per - 1) / c.rows_per);
    return (b + 7) / 8 * 8;
}
// Pass 1 of a join: R and S are its two segments (tiles numbered R first).
// The pass-1 histogram takes them from here, as plain launch arguments, and
// its first workgroup writes what later launches read from memory: the two
// segment descriptors (segs[0..1]), tile_begin[0..2] = {0, nt_r, nt_r + nt_s},
// and zero[0..nzero) cleared (the join's scan states).
struct Pass1 {
    const int32_t* rk;
    const int32_t* rr;
    const int32_t* sk;
    const int32_t* sr;
    uint32_t n_r, n_s;
    uint32_t nt_r, ntiles;
    uint64_t hist_s;  // first histogram entry of S: nt_r << bits
    PartSeg* segs;
    uint32_t* tile_begin;
    uint64_t* zero;
    uint64_t nzero;
    uint64_t* err_clear;  // the call's error word, cleared with the scan states (or nullptr)
    // counted pass 2: rows[tile * 2^bits_all + i] = tuples of the tile in final
    // partition i = hash & (2^bits_all - 1), esc[tile * kCountEsc + k] its
    // escapes (rows == nullptr: no counting)
    uint8_t* rows;
    uint32_t* esc;
    uint32_t bits_all;
    uint32_t pad;
};
Pass1 make_pass1(const int32_t* rk, const int32_t* rr, uint32_t n_r, const int32_t* sk, const int32_t* sr,
                 uint32_t n_s, uint32_t tile, uint32_t bits, PartSeg* segs, uint32_t* tile_begin, uint64_t* zero,
                 uint64_t nzero, uint64_t* err_clear);
// Pass-1 histogram (and the pass's set-up, see Pass1).
void part_hist_pass1(const Pass1& p1, const PassCfg& cfg, uint32_t* hist, Recorder& rec);
// Histogram of a later pass over the segments in memory; tile_seg: segment of
// every tile (nullptr: binary search over tile_begin).
void part_hist(const PartSeg* segs, const uint32_t* tile_begin, const uint32_t* tile_seg, uint32_t nseg,
               uint32_t grid, const PassCfg& cfg, uint32_t* hist, Recorder& rec);
// Partition boundaries of a one-segment pass (R only, segment at position 0):
// starts[p] for p < 2^bits from the pass's histogram scan, starts[2^bits] = n.
void part_starts(const uint32_t* hist_scan, uint32_t ntiles, uint32_t bits, uint32_t n, uint32_t* starts,
                 Recorder& rec);
// `side`: extra workgroups appended to the grid that run the next step's setup
// (hj_side.h: the pass-2 segment table or the join plan).
struct SideJob;
// rsv (counted pass 2): offsets from the totals and cursors instead of hist_scan.
void part_scatter(const PartSeg* segs, const uint32_t* tile_begin, const uint32_t* tile_seg, uint32_t nseg,
                  uint32_t grid, const PassCfg& cfg, const uint32_t* hist_scan, int32_t* key_out,
                  int32_t* rid_out, const SideJob& side, Recorder& rec, const Reserve* rsv = nullptr);

// ---- phj_join.hip ----
constexpr uint32_t kJoinBlock = 512;
constexpr uint32_t kJoinWaves = kJoinBlock / 64;
constexpr uint32_t kJoinSub = 4608;     // S tuples per probe round of a work item (9 per lane)
constexpr uint32_t kJoinChunk = 2 * kJoinSub;  // S tuples per work item (probed kJoinSub at a time)
// R tuples per HBM-table build item: 8 rounds of a workgroup, or 64 in a
// partition of more than kOvfBigPart tuples.  Small items keep the build's
// latency low; in a large partition, which is large because a key is heavy as
// often as not, each item's pushes of that key end in one exchange on its
// slot, and those exchanges serialize.
constexpr uint32_t kOvfChunk = 2048;
constexpr uint32_t kOvfChunkBig = 16384;
constexpr uint32_t kOvfBigPart = 1u << 16;
constexpr uint32_t kOvfGrid = 2048;  // workgroups of the HBM-table build launches (8 per CU)
__host__ __device__ inline uint32_t ovf_chunk(uint32_t r_len) { return r_len > kOvfBigPart ? kOvfChunkBig : kOvfChunk; }
constexpr uint32_t kMaxLdsCap = 8192;   // largest R partition held in LDS
// R tuples per thread of the LDS build (a kernel template argument: the build
// keeps them in registers), by lds_cap class.
constexpr uint32_t kRptSmall = 4, kRptMid = 9, kRptLarge = kMaxLdsCap / kJoinBlock;
inline uint32_t join_rpt(uint32_t lds_cap) {
    return lds_cap <= kRptSmall * kJoinBlock ? kRptSmall : (lds_cap <= kRptMid * kJoinBlock ? kRptMid : kRptLarge);
}
struct JoinPlanOut {
    PartPair* pairs;       // [P]
    uint32_t* item_begin;  // [P + 1] exclusive scan of work items per partition
    uint32_t* ovf_begin;   // [P + 1] exclusive scan of HBM-table build chunks per partition
    ItemRec* item_rec;     // [join_grid] every work item's R range and S chunk
    uint32_t* ovf_part;    // [ovf_grid] partition of every HBM-table build chunk
};
// The join plan (final partition table, work-item and overflow-chunk scans and
// maps) runs as a side job of the last scatter (hj_side.h); its state needs
// plan_state_words(2^total_bits) words that are zero when it starts.
size_t plan_state_words(uint32_t P);
// Upper bounds of the HBM-table build items and of the join work items.
uint32_t ovf_grid(uint32_t P, uint64_t n_r);
uint32_t join_grid(uint32_t P, uint64_t n_s);  // (a multiple of 8 kItemGroup)
constexpr uint32_t kItemGroup = 16;  // consecutive join items dealt to one XCD
// Dynamic LDS bytes of the join kernels for a given lds_cap.
size_t join_lds_bytes(uint32_t lds_cap, bool write);
size_t part_scatter_lds_bytes(uint32_t bits, uint32_t tile);
// hot: where the build records its hot keys (zeroed before); heavy: the
// one-pass queue (nullptr for count -> scan -> write), whose `wait` it sets.
// clear == false: the tables were cleared by the last scatter (Reserve::ovf_table).
void join_ovf_build(const PartPair* pairs, const uint32_t* ovf_begin, const uint32_t* ovf_part, uint32_t P,
                    uint32_t grid, const int32_t* rk, uint64_t* ovf_table, uint32_t* ovf_next, HotKeys* hot,
                    HeavyQueue* heavy, Recorder& rec, bool clear = true);
// item_begin/item_rec come from the join plan (JoinPlanOut).
void join_count(const PartPair* pairs, const uint32_t* item_begin, const ItemRec* item_rec, uint32_t P,
                uint32_t grid,
                const int32_t* rk, const int32_t* sk, uint32_t lds_cap, const uint64_t* ovf_table,
                const uint32_t* ovf_next, const HotKeys* hot, uint64_t* wave_cnt, bool nt_s, Recorder& rec);
void join_write(const PartPair* pairs, const uint32_t* item_begin, const ItemRec* item_rec, uint32_t P,
                uint32_t grid,
                const int32_t* rk, const int32_t* rr, const int32_t* sk, const int32_t* sr,
                uint32_t lds_cap, const uint64_t* ovf_table, const uint32_t* ovf_next,
                const uint64_t* wave_base, uint64_t* total, int32_t* out_r, int32_t* out_s,
                const HotKeys* hot, uint64_t capacity, HeavyQueue* heavy, bool nt_s, Recorder& rec);
// nt_s: S chunks read with non-temporal loads (LDS-table items).
// wave_base == nullptr selects the one-pass write: `total` must be zero on entry
// and ends as the number of pairs; `heavy` (one-pass only, zeroed before the
// HBM-table build, or nullptr) takes the heavy S tuples of HBM-table
// partitions that span several kHelpChunk-row chunks.  `hot`: the keys the
// HBM-table build recorded (their S tuples skip the chain walk).
// Writes zero to *d_count (joins with an empty side) and clears the call's
// error word (rec.err_clear).
void write_zero_count(uint64_t* d_count, Recorder& rec);

// ---- direct joins (no partitioning: R fits one LDS table) ----
// One job of the multi-job direct kernel.  Work item = (job, chunk of
// kJoinChunk S tuples); items of job j are [item0, item0 + ceil(n_s / chunk)).
struct DirectJob {
    const int32_t* rk;
    const int32_t* rr;
    const int32_t* sk;
    const int32_t* sr;
    int32_t* out_r;
    int32_t* out_s;
    uint64_t capacity;
    uint64_t* count;  // running total of the job's pairs (zeroed by direct_zero)
    uint32_t n_r, n_s, item0, pad;
};
// Writes one job descriptor and item map from kernel arguments, zeroes the
// job's count and clears the call's error word (rec.err_clear) (single join).
void direct_setup_one(DirectJob* job, uint32_t* item_job, const DirectJob& j, uint32_t nitems, Recorder& rec);
void direct_zero(const DirectJob* jobs, uint32_t njobs, Recorder& rec);
// lds_cap >= every job's n_r (<= kMaxLdsCap).
void direct_join(const DirectJob* jobs, const uint32_t* item_job, uint32_t nitems, uint32_t lds_cap,
                 Recorder& rec);

}  // namespace hj
