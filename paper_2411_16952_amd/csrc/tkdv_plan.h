// Host precompute (alpha*, proposal variances, rejection constant) -- FP64.
#pragma once

#include "../../include/tkdv.h"

namespace tkdv {

double plan_F(int K, double beta_p, double alpha);
bool plan_alpha_root_exists(int K, double beta_p);
int plan_alpha_star(int K, double beta_p, double *out);
int plan_point_host(const tkdv_point *pt, int proposal, int n_random, tkdv_plan *out);
double plan_log_ratio(const tkdv_point *pt, const tkdv_plan *pl, const double *xhat);

}  // namespace tkdv
