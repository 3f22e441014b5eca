// Planner internals of libmj: device time model and cost formulas.
#pragma once
#include <stdint.h>

#include "mj.h"

namespace mj {

struct DeviceModel {
    double stream_gbs;
    double probe_ps;
    double atomic_ps;
    double launch_us;
    double lds_ps;
    double list_ps;
};

// star plans: R's distinct B values must fit one workgroup's LDS array
// (the kernels' STAR_GROUPS), T's table one workgroup's LDS stage (T's
// one-bucket table is also built by a single workgroup: at 2^22 tuples
// that build alone took about 20 ms), and the star cascade's intermediate
// one chunk of the workspace
constexpr uint64_t STAR_PLAN_MAX_R = 4096;
constexpr uint64_t STAR_PLAN_MAX_T = 4096;
constexpr uint64_t STAR_PLAN_MAX_I = uint64_t(1) << 28;
inline bool star_plan_fits(const mj_plan_t& p) {
    return p.n_r <= STAR_PLAN_MAX_R && p.n_t <= STAR_PLAN_MAX_T;
}

// the degree-oriented cyclic join pays for its orientation pass (about
// 0.4 ms of extra launches) when the relation is large and its wedges dense:
// |R |x| S| = sum of squared degrees at least ORIENT_MIN_WEDGES per tuple
// (degree skew), and at least ORIENT_MIN_N tuples; both fitted on measured
// times of both algorithms over generated G(n, m), Chung-Lu and R-MAT
// graphs of 10^3 to 2 x 10^6 edges
constexpr uint64_t ORIENT_MIN_N = 32768;
constexpr uint64_t ORIENT_MIN_WEDGES = 64;
inline bool orient_pays(const mj_plan_t& p) {
    return p.n_r >= ORIENT_MIN_N && p.join2_size >= ORIENT_MIN_WEDGES * p.n_r;
}

DeviceModel default_model();
int analytic_plan(int kind, mj_plan_t& p, int num_cu, const DeviceModel& m);

double cost_linear_tuples(double R, double S, double T, double M);
double cost_cascade_tuples(double I);
double linear_break_even_M(double R, double S, double T, double I);
double cost_cyclic_tuples(double R, double S, double T, double M, double H);
double cyclic_optimal_H(double R, double S, double T, double M);
double cost_cyclic_min(double R, double S, double T, double M);
double join2_uniform_estimate(double R, double S, double d);
double branch_hit_probability(double g3, double d);

double model_linear_3way_ms(const DeviceModel& m, double R, double S, double T);
double model_linear_cascade_ms(const DeviceModel& m, double R, double S, double T, double I);
double model_star_ms(const DeviceModel& m, double R, double S, double T);
double model_star_cascade_ms(const DeviceModel& m, double R, double S, double T, double I);
double model_slarge_ms(const DeviceModel& m, double R, double S, double T, uint32_t lr, uint32_t lt);
bool slarge_buckets(const DeviceModel& m, uint64_t n_r, uint64_t n_s, uint64_t n_t, uint32_t& lr,
                    uint32_t& lt, double* ms);
double model_cyclic_ms(const DeviceModel& m, double R, double S, double T, double I, double share);
double model_cyclic_cascade_ms(const DeviceModel& m, double R, double S, double T, double I);

}  // namespace mj
