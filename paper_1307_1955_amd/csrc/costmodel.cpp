// Per-step cost model of a join on MI355X (Section 4, Eq. 2-3) and the
// planner that evaluates it (HJ_AUTO).
//
// The paper sums, over a step series, each step's computation time, memory
// stall time and pipelined delay.  One GPU runs every step here, and a step is
// one kernel launch of the plan (engine.cpp's launch sequence):
//     T = sum over launches k of  D + d + max(M_k, W_k)
// D: delay of a dependent launch behind the previous kernel; d: a kernel's
// fixed ramp-up and drain; M_k: the launch's algorithmic bytes over the
// bandwidth of its access pattern (streaming read, scatter whose bandwidth
// grows with the run length tile / 2^bits, random table lines served from the
// caches or from HBM); W_k: rounds of resident workgroups times one
// workgroup's duration (the latency-bound join items; for the partitioning
// tiles the first round's and a share q_part of every later round's, as
// later rounds overlap the ones before).  The constants come
// from per-kernel HIP-event times of a grid of joins on MI355X (generated
// include calib_mi355x.inc; the Python twin paper_1307_1955_amd/costmodel.py
// fits them and is kept equal to this file by a test).
#include <algorithm>
#include <cmath>

#include "../../include/hj.h"
#include "engine.h"
#include "hj_internal.h"

namespace hj {
namespace eng {

namespace {

#include "calib_mi355x.inc"

constexpr double kCus = 256;
constexpr double kLdsPerCu = 160.0 * 1024;
constexpr double kChunk = kJoinChunk;
constexpr double kShjTileD = kShjTile;
constexpr double kOvfGridD = kOvfGrid;

double part_block(uint32_t tile) { return tile >= 4096 ? 512 : 256; }

double scatter_slots(uint32_t bits, uint32_t tile) {
    const double P = std::ldexp(1.0, (int)bits);
    const double Pp = std::max(P, 64.0);
    const double lds = 4 * (2 * Pp + 16) + 8.0 * tile;
    const double by_lds = std::floor(kLdsPerCu / lds);
    const double by_threads = std::floor(2048 / part_block(tile));
    return kCus * std::max(1.0, std::min(by_lds, by_threads));
}

double hist_slots(uint32_t tile) { return kCus * std::floor(2048 / part_block(tile)); }

// Join work items resident at once: workgroups per CU by LDS and by the waves
// the kernels' register budget allows (6 per SIMD, 4 with the largest build).
double join_slots(uint32_t cap) {
    const double lds = 4.0 * (cap + 128) + 8.0 * cap;
    const double by_waves = (join_rpt(cap) > kRptMid ? 4.0 : 6.0) * 4.0 / kJoinWaves;
    return kCus * std::max(1.0, std::min(std::floor(kLdsPerCu / (lds + 1024)), std::floor(by_waves)));
}

double nonempty(double mean) { return mean < 30 ? 1.0 - std::exp(-mean) : 1.0; }

// Change of a random access's cost with the table size (1 up to base bytes).
double table_factor(double table_bytes, double gamma, double base = 1048576.0) {
    return std::pow(std::max(table_bytes, base) / base, gamma);
}

double rounds(double items, double slots) { return std::ceil(std::max(items, 1.0) / slots); }

// (a^p + b^p)^(1/p): max(a, b) as p grows, more than it when a and b are close.
double smooth_max(double a, double b, double p) {
    const double m = std::max(a, b);
    if (m <= 0) return 0;
    return m * std::pow(std::pow(a / m, p) + std::pow(b / m, p), 1.0 / p);
}

// extra: bytes beyond the tuples' (a counted pass 2's count rows); bins: the
// counters a counted pass 2's histogram tile clears, counts and packs
// Latency term of a partitioning launch: the first round of tiles, then a
// share q_part of each later round (rounds overlap).
double part_lat(double rounds, double per_tile) { return per_tile * (1.0 + (rounds - 1.0) * k_q_part); }

double hist_s(double n, double tiles, uint32_t tile, double extra, double bins) {
    if (tiles == 0) return k_d_kernel;
    const double per_tile = k_t_hist_tile * tile / 8192.0 + k_t_count_bin * bins;
    return k_d_kernel + smooth_max((4.0 * n + extra) / k_bw_hist,
                                   part_lat(rounds(tiles, hist_slots(tile)), per_tile), k_p_part);
}

// counted: a counted pass 2's scatter (count sums beside pass 1, reservations in pass 2)
double scatter_s(double n, double tiles, uint32_t tile, uint32_t bits, double extra, bool counted) {
    if (tiles == 0) return k_d_kernel;
    const double run = tile / std::ldexp(1.0, (int)bits);
    const double bw = k_bw_scatter * run / (run + k_run_half);
    const double per_tile = k_t_scatter_tile * tile / 8192.0 + (counted ? k_t_reserve : 0.0);
    return k_d_kernel + smooth_max((16.0 * n + extra) / bw,
                                   part_lat(rounds(tiles, scatter_slots(bits, tile)), per_tile), k_p_part);
}

double scan_s(double entries) { return k_d_kernel + entries * k_t_scan_entry; }

// f: the kernel's work-item latency against the write pass (k_f_count, k_f_1pass, or 1)
double join_s(double items, double r, double s, uint32_t cap, bool hbm, double bytes, double f) {
    const double lat = f * (hbm ? k_l_hbm0 + k_l_hbm_s * s : k_l_join0 + k_l_join_r * r + k_l_join_s * s);
    return k_d_kernel + smooth_max(bytes / k_bw_join, rounds(items, join_slots(cap)) * lat, k_p_join);
}

}  // namespace

double model_seconds(const Plan& pl, uint64_t n_r_, uint64_t n_s_, double m) {
    const double n_r = (double)n_r_, n_s = (double)n_s_, n = n_r + n_s;
    const double gap = k_d_gap, d = k_d_kernel;
    if (n_r_ == 0 || n_s_ == 0) return gap + d;
    double t = 0;
    int nl = 0;
    if (!pl.phj) {
        const double slots = (double)shj_slots(n_r_);
        const double tb = 8 * slots;
        const double ins = k_t_ins * table_factor(tb, k_gamma_ins);
        const double probe = k_t_probe * table_factor(tb, k_gamma_probe);
        const double b_floor = k_t_bround * table_factor(tb, k_gamma_bround, 32768.0);
        const double p_floor = k_t_pround * table_factor(tb, k_gamma_pround, 32768.0);
        const double probe_s = std::max(n_s * probe, p_floor);
        const double write_s = std::max(n_s * probe + m * k_t_match, p_floor);
        t += d + 8 * slots / k_bw_fill;            // fill
        t += d + std::max(n_r * ins, b_floor);     // build
        nl += 2;
        if (pl.one_pass) {
            t += d;            // zero the count and the queue
            t += d + write_s;  // write
            nl += 2;
        } else {
            t += d + probe_s;                             // count
            t += d;                                       // zero the scan state
            t += scan_s(4 * std::ceil(n_s / kShjTileD));  // scan of the per-wave counts
            t += d + write_s;                             // write
            nl += 4;
        }
        return t + nl * gap;
    }
    if (pl.passes == 0) {
        const double items = std::ceil(n_s / kChunk);
        t += d;  // setup
        t += join_s(items, n_r, std::min(n_s, kChunk), pl.lds_cap, false, 8 * n + 8 * m, 1.0);
        return t + 2 * gap;
    }
    const uint32_t tile = pl.tile, b1 = pl.b1, b2 = pl.passes == 2 ? pl.b2 : 0;
    const double P = std::ldexp(1.0, (int)(b1 + b2)), P1 = std::ldexp(1.0, (int)b1);
    const double tiles1 = std::ceil(n_r / tile) + std::ceil(n_s / tile);
    const bool counted = counted_pass2(pl.passes, b1, b2);
    const double r_part = n_r / P, s_part = n_s / P;
    const bool hbm = r_part > pl.lds_cap;
    const double ovf_r = hbm ? n_r : 0;
    const bool clears = counted && counted_clears_tables(b2);  // the pass-2 scatter clears the HBM tables
    const double rows = counted ? tiles1 * P : 0.0;  // 8-bit count rows: histogram writes, sums beside the scatter read
    t += hist_s(n, tiles1, tile, rows, counted ? P : 0.0) + scan_s(tiles1 * P1) +
         scatter_s(n, tiles1, tile, b1, rows, counted);
    nl += 3;
    if (pl.passes == 2) {
        const double seg = n / (2 * P1);
        const double tiles2 = seg > 0 ? 2 * P1 * std::max(1.0, std::ceil(seg / tile)) : 0;
        if (!counted) {
            t += hist_s(n, tiles2, tile, 0.0, 0.0) + scan_s((n / tile + 2 * P1) * std::ldexp(1.0, (int)b2));
            nl += 2;
        }
        t += scatter_s(n, tiles2, tile, b2, clears ? 16 * ovf_r : 0.0, counted);
        nl += 1;
    }
    const double items = P * nonempty(r_part) * nonempty(s_part) * std::max(1.0, std::ceil(s_part / kChunk));
    const double grid = P + std::ceil(n_s / kChunk);
    const double s_item = std::min(std::max(s_part, 1.0), kChunk);
    const double r_item = std::min(r_part, (double)pl.lds_cap);
    if (!clears) {
        t += d + 16 * ovf_r / k_bw_fill;  // clear the HBM tables
        nl += 1;
    }
    t += d;  // build them: inserts, or rounds of items of ovf_chunk() tuples
    if (hbm) {
        const double chunk = r_part > kOvfBigPart ? kOvfChunkBig : kOvfChunk;
        const double ovf_items = P * std::ceil(r_part / chunk);
        const double ovf_rounds = std::ceil(ovf_items / std::min(kOvfGridD, 8 * kCus));
        t += std::max(ovf_r * k_t_ovf_insert, ovf_rounds * std::ceil(std::min(r_part, chunk) / 256) * k_l_ovf_round);
    }
    nl += 1;
    if (!pl.one_pass) {
        t += join_s(items, r_item, s_item, pl.lds_cap, hbm, 4 * n, k_f_count);
        t += scan_s(8 * grid);
        t += join_s(items, r_item, s_item, pl.lds_cap, hbm, 8 * n + 8 * m, 1.0);
        nl += 3;
    } else {
        t += join_s(items, r_item, s_item, pl.lds_cap, hbm, 8 * n + 8 * m, k_f_1pass);
        nl += 1;
    }
    return t + nl * gap;
}

// HJ_AUTO: the plan with the least modelled time among SHJ, the direct LDS join
// (|R| <= 8192) and PHJ in one or two radix passes around ~4096 R tuples per
// partition.  The partitioning tile is the caller's, else the measured size
// rule (default_tile): between the two tiles the model cannot see which pass
// loses by shorter runs (pass 1 reads the inputs cold; 16M x 16M ran 9% slower
// with 4096-tuple tiles, which the model priced faster).  Hash, lds_cap and
// flags are the caller's.  The output size is taken as |S|
// (one match per probe tuple), the same for every candidate.
void auto_params(uint64_t n_r, uint64_t n_s, hj_params* p) {
    const hj_params base = *p;
    const double m = (double)n_s;
    double best_t = 1e300;
    hj_params best = base;
    best.algo = HJ_PHJ;
    best.passes = 1;
    best.bits[0] = 1;
    best.bits[1] = 0;
    auto consider = [&](const hj_params& q) {
        Plan pl;
        const hj_status st = check_params(&q, n_r, n_s, &pl);
        if (st != HJ_OK) return;
        const double t = model_seconds(pl, n_r, n_s, m);
        if (t < best_t) {
            best_t = t;
            best = q;
        }
    };
    hj_params q = base;
    q.algo = HJ_SHJ;
    q.passes = 0;
    q.bits[0] = q.bits[1] = 0;
    consider(q);
    q.algo = HJ_PHJ;
    if (n_r <= kMaxLdsCap) consider(q);  // passes 0: one LDS table
    uint32_t B = 0;
    while (B < kMaxRadixBits && (n_r >> B) > 4096) ++B;
    for (uint32_t b = (B > 2 ? B - 2 : 1); b <= std::min(B + 2, kMaxRadixBits); ++b) {
        {
            q.tile = base.tile;  // 0: the size rule
            if (b <= 13) {
                q.passes = 1;
                q.bits[0] = b;
                q.bits[1] = 0;
                consider(q);
            }
            if (b >= 2) {
                q.passes = 2;
                for (uint32_t b1 = std::max(1u, b / 2 - 1); b1 <= std::min(13u, b / 2 + 2); ++b1) {
                    if (b - b1 < 1 || b - b1 > 13) continue;
                    q.bits[0] = b1;
                    q.bits[1] = b - b1;
                    consider(q);
                }
            }
        }
    }
    *p = best;
    p->tile = base.tile ? base.tile : best.tile;
}

}  // namespace eng
}  // namespace hj
