// Analytic planner of libmj: the paper's cost formulas (tuples read onto the
// chip) and an MI355X time model built on them, used to choose between the
// three-way join and the cascade and to pick bucket counts and shares.
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "mj.h"
#include "mj_host.h"
#include "mj_plan_model.h"

namespace mj {

// ---------------------------------------------------------- paper formulas
// Sec. 4.2: R and S are read once, T once per partition of R (|R|/M of them).
double cost_linear_tuples(double R, double S, double T, double M) { return R + S + R * T / M; }

// Example 3: the cascade writes its intermediate and reads it back.
double cost_cascade_tuples(double I) { return 2.0 * I; }

// Example 3 solved for M: the smallest on-chip capacity for which the
// three-way join reads fewer tuples than the cascade moves.
double linear_break_even_M(double R, double S, double T, double I) {
    const double room = 2.0 * I - R - S;
    return room <= 0.0 ? INFINITY : R * T / room;
}

// Sec. 5.2: |R| + H|S| + G|T| with G H = |R| / M.
double cost_cyclic_tuples(double R, double S, double T, double M, double H) {
    return R + H * S + (R / (M * H)) * T;
}
double cyclic_optimal_H(double R, double S, double T, double M) { return std::sqrt(R * T / (M * S)); }
double cost_cyclic_min(double R, double S, double T, double M) {
    return R + 2.0 * std::sqrt(R * S * T / M);
}

// Sec. 6.3: |R join S| under uniform keys with d distinct values.
double join2_uniform_estimate(double R, double S, double d) { return R * S / d; }

// App. A: branch hit probability of the S.C = T.C test with g3 buckets.
double branch_hit_probability(double g3, double d) { return g3 / d; }

// ----------------------------------------------------------- time model
// Device constants, calibrated on MI355X with the benchmark workloads:
//   stream_gbs  bandwidth the partition/scan kernels reach (GB/s)
//   probe_ps    amortised cost of one random table probe (ps)
//   atomic_ps   amortised cost of one random 64-bit global atomic (ps)
//   launch_us   fixed cost per kernel launch (us)
//   lds_ps      amortised cost of one LDS probe in the cyclic join (ps)
//   list_ps     amortised cost of one streamed list element (ps)
DeviceModel default_model() {
    DeviceModel m;
    m.stream_gbs = 1900.0;
    m.probe_ps = 21.0;
    m.atomic_ps = 24.0;
    m.launch_us = 6.0;
    m.lds_ps = 8.0;
    m.list_ps = 30.0;
    return m;
}

// Linear three-way join: partitions (R, S: 16 B/tuple each pass incl. the
// histogram read; T: 12 B), T's tables, one table probe per S tuple, one
// LDS probe + one count atomic per R tuple, about 20 launches.
double model_linear_3way_ms(const DeviceModel& m, double R, double S, double T) {
    const double bytes = 24.0 * (R + S) + 16.0 * T + 16.0 * (R + S);
    const double t = bytes / (m.stream_gbs * 1e9) + (S * m.probe_ps + R * m.atomic_ps) * 1e-12 +
                     20.0 * m.launch_us * 1e-6;
    return t * 1e3;
}

// Cascade: the same partitions, R grouped by B, the scan over S, the
// intermediate written and read (8 B each way per pair), one table probe
// and one count atomic per pair.
double model_linear_cascade_ms(const DeviceModel& m, double R, double S, double T, double I) {
    const double bytes = 24.0 * (R + S) + 16.0 * T + 12.0 * R + 20.0 * S + 16.0 * I;
    const double t = bytes / (m.stream_gbs * 1e9) + I * (m.probe_ps + m.atomic_ps) * 1e-12 +
                     26.0 * m.launch_us * 1e-6;
    return t * 1e3;
}

// Star three-way join: one-bucket tables of R's B and T's C (a partition
// pass and a table build each), one pass over S with two probes of
// L2-resident tables per tuple, the per-block sums, a pass over R.
double model_star_ms(const DeviceModel& m, double R, double S, double T) {
    const double bytes = 8.0 * S + 28.0 * (R + T);
    const double t = bytes / (m.stream_gbs * 1e9) + 2.0 * S * m.lds_ps * 1e-12 +
                     16.0 * m.launch_us * 1e-6;
    return t * 1e3;
}

// Binary star cascade: the same tables, R grouped by B, two passes over S
// (count, then expand I with a prefix sum between), I written and read
// (8 B each way per pair) with one probe of T per pair.
double model_star_cascade_ms(const DeviceModel& m, double R, double S, double T, double I) {
    const double bytes = 28.0 * S + 16.0 * I + 40.0 * (R + T);
    const double t = bytes / (m.stream_gbs * 1e9) + (2.0 * S + I) * m.lds_ps * 1e-12 +
                     26.0 * m.launch_us * 1e-6;
    return t * 1e3;
}

// S-largest form of the linear join (Sec. 4, after Algorithm 1).  Per S
// tuple: the partition by the pair (bucket of B, bucket of C) and one pass
// of the cell kernel (an LDS probe of T_j's table, an LDS probe of R_i's B
// values, an LDS add).  Both were measured on MI355X over star schemas with
// 2^24..2^26 S tuples and R, T of 2^12..2^22 tuples:
//   partition, per S tuple: 7.5 ps with at most 2^10 cells, 12.8 ps with
//     2^11, 16.8 ps with 2^12 (more buckets than the scatter's LDS stage
//     holds at full speed);
//   cell pass, per S tuple: 5.5 ps while T_j (about |T| / L_T tuples) fits
//     the 4096-slot LDS stage, 4 ps more per doubling of T_j beyond 2048
//     tuples (its probes go to L2 and beyond).
// R's parts hold about 1024 B values each (the table's 4096 slots staged
// in LDS stay at load 1/4 or less under the hash's imbalance); R and T are
// read, tabled and partitioned at stream rate, and each R tuple probes the
// sums once.
double slarge_part_ps(uint32_t bits) { return bits <= 10 ? 7.5 : bits == 11 ? 12.8 : 16.8; }
double slarge_cell_ps(double t_part) {
    return t_part <= 2048.0 ? 5.5 : 5.5 + 4.0 * std::log2(t_part / 2048.0);
}
double model_slarge_ms(const DeviceModel& m, double R, double S, double T, uint32_t lr, uint32_t lt) {
    const double bytes = 40.0 * R + 16.0 * T;
    const double t = bytes / (m.stream_gbs * 1e9) +
                     S * (slarge_part_ps(lr + lt) + slarge_cell_ps(T / double(1u << lt))) * 1e-12 +
                     R * m.atomic_ps * 1e-12 + 20.0 * m.launch_us * 1e-6;
    return t * 1e3;
}

// Bucket counts of the S-largest plan: L_R = 2^lr parts of R of about 1024
// tuples, and the L_T = 2^lt (lr + lt <= 12) the model above prefers.
// Returns false when R needs more than 2^12 parts.
constexpr uint32_t SLARGE_MAX_BITS = 12;   // cells: one partition pass's bucket limit
bool slarge_buckets(const DeviceModel& m, uint64_t n_r, uint64_t n_s, uint64_t n_t, uint32_t& lr,
                    uint32_t& lt, double* ms) {
    lr = ceil_log2((n_r + 1023) / 1024);
    lt = 0;
    if (lr > SLARGE_MAX_BITS) return false;
    double best = INFINITY;
    for (uint32_t k = 0; lr + k <= SLARGE_MAX_BITS; ++k) {
        const double t = model_slarge_ms(m, (double)n_r, (double)n_s, (double)n_t, lr, k);
        if (t < best) { best = t; lt = k; }
    }
    if (ms) *ms = best;
    return true;
}

// Cyclic join: three sorts (8 passes of 24 B/tuple), the run indexes, and
// the intersection work, bounded by the wedges the cascade would
// materialise (I); `share` slices hub lists and adds a list search per
// slice and S tuple of hub groups (taken as a fraction of S).
double model_cyclic_ms(const DeviceModel& m, double R, double S, double T, double I,
                       double share) {
    const double bytes = 8.0 * 24.0 * (R + S + T) + 40.0 * (R + S + T);
    const double inter = std::min(I, 64.0 * std::sqrt(I) * std::sqrt(std::max(1.0, S)));
    const double t = bytes / (m.stream_gbs * 1e9) + inter * m.list_ps * 1e-12 +
                     share * 0.05 * S * 20.0 * m.probe_ps * 1e-12 + 90.0 * m.launch_us * 1e-6;
    return t * 1e3;
}

// Cyclic cascade: the wedges are materialised and each is checked against T.
double model_cyclic_cascade_ms(const DeviceModel& m, double R, double S, double T, double I) {
    const double bytes = 8.0 * 24.0 * T + 24.0 * (R + S) + 16.0 * I;
    const double t = bytes / (m.stream_gbs * 1e9) + I * 3.0 * m.probe_ps * 1e-12 +
                     40.0 * m.launch_us * 1e-6;
    return t * 1e3;
}

int analytic_plan(int kind, mj_plan_t& p, int num_cu, const DeviceModel& m) {
    (void)num_cu;
    p.seed = 0x1B873593u;
    const double R = (double)p.n_r, S = (double)p.n_s, T = (double)p.n_t;
    const double I = (double)p.join2_size;
    if (kind == MJ_LINEAR) {
        // b-buckets: about 16K S tuples per W table; c-buckets: about 32K T
        // tuples per multiplicity table (at most 2^10 of either)
        p.log2_nb = std::min<uint32_t>(10, ceil_log2((p.n_s + 16383) / 16384));
        p.log2_nc = std::min<uint32_t>(10, ceil_log2((p.n_t + 32767) / 32768));
        p.est_ms_3way = model_linear_3way_ms(m, R, S, T);
        p.est_ms_cascade = model_linear_cascade_ms(m, R, S, T, I);
        p.est_ms_star = star_plan_fits(p) ? model_star_ms(m, R, S, T) : 0.0;
        p.est_ms_star_cascade = star_plan_fits(p) && p.join2_size <= STAR_PLAN_MAX_I
                                    ? model_star_cascade_ms(m, R, S, T, I) : 0.0;
    } else {
        // share on A (the least number of slices of a hub list): the
        // candidate of {1, 2, ..., 32} the time model prefers
        double best = INFINITY;
        uint32_t best_k = 0;
        for (uint32_t k = 0; k <= 5; ++k) {
            const double t = model_cyclic_ms(m, R, S, T, I, double(1u << k));
            if (t < best) { best = t; best_k = k; }
        }
        p.log2_share = best_k;
        p.log2_nb = std::min<uint32_t>(10, ceil_log2((p.n_s + 32767) / 32768));
        p.log2_nc = std::min<uint32_t>(10, ceil_log2((p.n_t + 32767) / 32768));
        p.est_ms_3way = best;
        p.est_ms_cascade = model_cyclic_cascade_ms(m, R, S, T, I);
    }
    p.algo = p.est_ms_cascade < p.est_ms_3way ? MJ_ALGO_CASCADE : MJ_ALGO_3WAY;
    if (kind == MJ_LINEAR) {
        // the star plans (when eligible) compete with the one chosen so far
        double best = std::min(p.est_ms_3way, p.est_ms_cascade);
        if (p.est_ms_star > 0.0 && p.est_ms_star < best) { p.algo = MJ_ALGO_STAR; best = p.est_ms_star; }
        if (p.est_ms_star_cascade > 0.0 && p.est_ms_star_cascade < best) {
            p.algo = MJ_ALGO_STAR_CASCADE;
            best = p.est_ms_star_cascade;
        }
        // S the largest relation and R or T too large for the star plans
        // (Sec. 4, after Algorithm 1).  Hashed tables only: with dense keys
        // the direct-indexed path is cheaper still.
        uint32_t lr = 0, lt = 0;
        double t_sl = 0.0;
        const bool eligible = !(p.flags & MJ_PLAN_DENSE_KEYS) && !star_plan_fits(p) &&
                              p.n_s >= 4 * std::max(p.n_r, p.n_t) && p.a_domain > 0 &&
                              p.a_domain <= (1u << 24) && slarge_buckets(m, p.n_r, p.n_s, p.n_t, lr, lt, &t_sl);
        p.est_ms_slarge = eligible ? t_sl : 0.0;
        if (eligible && p.est_ms_slarge < best) {
            p.algo = MJ_ALGO_SLARGE;
            p.log2_nb = lr;
            p.log2_nc = lt;
        }
    }
    return MJ_OK;
}

}  // namespace mj

// ------------------------------------------------------------- C ABI
extern "C" int mj_cost_model(int which, const double* args, int nargs, double* out) {
    using namespace mj;
    if (!args || !out) return MJ_ERR_INVALID_ARG;
    auto need = [&](int k) { return nargs >= k; };
    switch (which) {
        case MJ_COST_LINEAR_TUPLES:
            if (!need(4)) return MJ_ERR_INVALID_ARG;
            *out = cost_linear_tuples(args[0], args[1], args[2], args[3]); return MJ_OK;
        case MJ_COST_CASCADE_TUPLES:
            if (!need(1)) return MJ_ERR_INVALID_ARG;
            *out = cost_cascade_tuples(args[0]); return MJ_OK;
        case MJ_COST_LINEAR_BREAK_EVEN_M:
            if (!need(4)) return MJ_ERR_INVALID_ARG;
            *out = linear_break_even_M(args[0], args[1], args[2], args[3]); return MJ_OK;
        case MJ_COST_CYCLIC_TUPLES:
            if (!need(5)) return MJ_ERR_INVALID_ARG;
            *out = cost_cyclic_tuples(args[0], args[1], args[2], args[3], args[4]); return MJ_OK;
        case MJ_COST_CYCLIC_OPTIMAL_H:
            if (!need(4)) return MJ_ERR_INVALID_ARG;
            *out = cyclic_optimal_H(args[0], args[1], args[2], args[3]); return MJ_OK;
        case MJ_COST_CYCLIC_MIN:
            if (!need(4)) return MJ_ERR_INVALID_ARG;
            *out = cost_cyclic_min(args[0], args[1], args[2], args[3]); return MJ_OK;
        case MJ_COST_JOIN2_UNIFORM:
            if (!need(3)) return MJ_ERR_INVALID_ARG;
            *out = join2_uniform_estimate(args[0], args[1], args[2]); return MJ_OK;
        case MJ_COST_BRANCH_HIT:
            if (!need(2)) return MJ_ERR_INVALID_ARG;
            *out = branch_hit_probability(args[0], args[1]); return MJ_OK;
        default:
            return MJ_ERR_INVALID_ARG;
    }
}

extern "C" int mj_slarge_buckets(uint64_t n_r, uint64_t n_s, uint64_t n_t, uint32_t* log2_nb,
                                 uint32_t* log2_nc, double* est_ms) {
    using namespace mj;
    if (!log2_nb || !log2_nc) return MJ_ERR_INVALID_ARG;
    uint32_t lr = 0, lt = 0;
    double ms = 0.0;
    if (!slarge_buckets(default_model(), n_r, n_s, n_t, lr, lt, &ms)) return MJ_ERR_INVALID_ARG;
    *log2_nb = lr;
    *log2_nc = lt;
    if (est_ms) *est_ms = ms;
    return MJ_OK;
}
