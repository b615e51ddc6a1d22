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

struct PlanArgs {
    const PlanPoint *pts;
    int n_items;        // points x starts
    int n_starts;
    uint32_t seed_lo, seed_hi;
    double *val;        // [n_items] objective at the final iterate
    double *xbest;      // [n_items][128] final iterate (unit vector)
    int *evals;         // [n_items] objective evaluations
};

hipError_t launch_plan_search(const PlanArgs &a, hipStream_t st);

}  // namespace tkdv
