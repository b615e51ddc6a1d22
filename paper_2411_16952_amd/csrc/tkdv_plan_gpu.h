// Multi-start search for the rejection constant on the GPU (step 1 of
// Sec. IV.B, the maximisation of Sec. IV.A): shared between the launcher in
// tkdv_plan_gpu.hip and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tkdv {

constexpr int kPlanWaves = 4;          // wavefronts (starts) per workgroup
constexpr int kPlanMem = 8;            // L-BFGS memory (pairs)
constexpr int kPlanMaxIter = 400;      // ascent iterations per start
constexpr int kPlanMaxBacktrack = 50;  // step halvings per line search
constexpr int kPlanStride = 256;       // doubles per start / final iterate (2 TKDV_KMAX)

// One point of the search: the objective is
//   phi(x^) = dt0 t + cH (pi/(3N)) amp^3 sum_j u~_j^3 [+ K log(1 + a t)]
// with t = sum_k k^2 s_k, u~ = Phi^T x^ on the N = 4K grid, amp = sqrt(2 E0/pi),
// dt0 = -beta'/K^2, cH = beta' (C3/C2)/(E0 K^2), a = alpha* beta'/K^3; the
// bracket is present for the Sigma proposal (sigma = 1).
struct PlanPoint {
    int K, N, sigma;
    uint32_t point_id;  // counter word of the random starts
    double dt0, cH, amp3, a;
};

// The learned mixture of a point (K <= 32), for the search of
// M_mix = sup f/q_mix: phi = log f - log q_mix with
//   log q_mix = LSE(log eps + lg(t), log(1 - eps) + log q_net),
//   lg(t) = lng - K log(1 + gc t) (the normalised g_Sigma),
//   log q_net = -logdetL0/2 + LSE_j(-K log qf_j) - log S,
//   qf_j = e^T A e + |g|^2, w = R_j^T x, g = Ginv V^T A w, e = w - V g.
struct PlanMix {
    double a[64];         // 1/d per coordinate
    double V[64][2];      // base rank-2 factor, rows = coordinates
    double gi[2][2];      // (I + V^T A V)^-1
    double cs[32], sn[32];  // cos, sin of 2 pi m/S
    double logdetL0, lng, log_eps, log_1m_eps, gc;
};

struct PlanArgs {
    const PlanPoint *pts;
    const PlanMix *mix;     // [points] or nullptr: the mixture objective
    const double *x_user;   // [points][n_user][kPlanStride] caller starts or nullptr
    int n_user;             // caller starts per point (items n_starts .. n_starts + n_user - 1)
    int n_items;        // points x (n_starts + n_user)
    int n_starts;       // generated starts per point
    uint32_t seed_lo, seed_hi;
    double *val;        // [n_items] objective at the final iterate
    double *xbest;      // [n_items][kPlanStride] final iterate (unit vector)
    int *evals;         // [n_items] objective evaluations
};

// max_K: the largest K among the points (at most kPlanStride / 2)
hipError_t launch_plan_search(const PlanArgs &a, int max_K, hipStream_t st);

}  // namespace tkdv
