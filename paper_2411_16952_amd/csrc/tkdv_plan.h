// Host precompute (alpha*, proposal variances, rejection constant) -- FP64.
#pragma once

#include "../../include/tkdv.h"

namespace tkdv {

double plan_F(int K, double beta_p, double alpha);
bool plan_alpha_root_exists(int K, double beta_p);
int plan_alpha_star(int K, double beta_p, double *out);
// alpha*, s_k^2, log_norm_g and, for C3/C2 = 0, the closed-form log M
// (M_source 0); otherwise log_M is left at 0 with M_source -1 (to be searched).
int plan_base_host(const tkdv_point *pt, int proposal, tkdv_plan *out);
int plan_point_host(const tkdv_point *pt, int proposal, int n_random, tkdv_plan *out);
double plan_log_ratio(const tkdv_point *pt, const tkdv_plan *pl, const double *xhat);

}  // namespace tkdv
