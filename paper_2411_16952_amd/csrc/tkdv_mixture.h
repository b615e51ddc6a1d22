// Host FP64 evaluation of the learned defensive mixture proposal (see the
// tkdv_mixture description in include/tkdv.h): density, its gradient on the
// sphere, and the tables the GPU kernels use.
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/tkdv.h"

namespace tkdv {

struct MixHost {
    int K = 0;
    uint64_t E = 0;  // component word w < E selects g_Sigma; eps = E 2^-32
    double eps = 0.0, log_eps = 0.0, log_1m_eps = 0.0;
    double alpha = 1.0, beta_p = 0.0, lng = 0.0;  // g_Sigma
    std::vector<double> a;                        // 1/d for each of the 2K coordinates
    std::vector<double> sqd;                      // sqrt(d)
    std::vector<double> V;                        // [2K][R]
    double Ginv[TKDV_MIX_R][TKDV_MIX_R] = {};     // (I + V^T D^-1 V)^-1
    double G[TKDV_MIX_R][TKDV_MIX_R] = {};
    double logdetL0 = 0.0;                        // log |D + V V^T|
    std::vector<double> cs, sn;                   // cos/sin(k phi_j): [S][K]

    // returns TKDV_OK or an error for a non-finite or singular mixture
    int init(const tkdv_point &pt, const tkdv_plan &sigma_plan, const tkdv_mixture &m);
    // w = R_phi_j^T x (shift by -phi_j) and back
    void rot_inv(int j, const double *x, double *w) const;
    void rot(int j, const double *w, double *x) const;
    // log q_net, log q_mix at a unit vector x; optional ambient gradient of log q_mix
    void log_q(const double *x, double *lnet, double *lmix, double *grad_lmix) const;
    // largest eigenvalue of G = I + V^T D^-1 V: max over the sphere of (x^T D^-1 x)/(x^T L0^-1 x)
    double kappa() const;
};

struct DevMix;

// Per-point device constants and tables of the mixture sampler (layout in
// DevMix); tab receives the point's tables, d.tab_off is left to the caller.
void mix_device_data(const MixHost &mh, DevMix &d, std::vector<uint8_t> &tab);

// Bound on the FP32 fast path's error in log q_mix for this mixture and
// synthesis arithmetic (input error of x^, the matrix-core products of y,
// FP32 rounding of the quadratic forms, the hardware log2/exp2 and the
// final combination).
double mix_window_extra(const MixHost &mh, int precision);

}  // namespace tkdv
