// Host FP64 mixture proposal: density (Woodbury form without cancellation),
// gradient on the sphere, and the rejection constant M_mix = sup f/q_mix.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

#include "tkdv_host_math.h"
#include "tkdv_internal.h"
#include "tkdv_mixture.h"
#include "tkdv_plan.h"

namespace tkdv {

int MixHost::init(const tkdv_point &pt, const tkdv_plan &sp, const tkdv_mixture &m)
{
    K = pt.K;
    if (m.K != K || !(m.eps > 0.0 && m.eps < 1.0)) return TKDV_E_ARG;
    // the component is chosen from one 32-bit word: weight E 2^-32 exactly
    E = (uint64_t)TKDV_MIX_S * (uint64_t)std::floor(m.eps * 4294967296.0 / TKDV_MIX_S);
    if (E == 0 || E >= (1ull << 32)) return TKDV_E_ARG;
    eps = std::ldexp((double)E, -32);
    log_eps = std::log(eps);
    log_1m_eps = std::log1p(-eps);
    alpha = sp.alpha_star;
    beta_p = pt.beta_p;
    const double K3 = (double)K * K * K;
    lng = 0.0;
    for (int k = 1; k <= K; ++k) lng += std::log1p(alpha * beta_p * (double)k * k / K3);
    a.assign(2 * K, 0.0);
    sqd.assign(2 * K, 0.0);
    V.assign(2 * K * TKDV_MIX_R, 0.0);
    double ldD = 0.0;
    for (int k = 0; k < K; ++k) {
        if (!std::isfinite(m.logd[k])) return TKDV_E_ARG;
        ldD += 2.0 * m.logd[k];
        a[k] = a[K + k] = std::exp(-m.logd[k]);
        sqd[k] = sqd[K + k] = std::exp(0.5 * m.logd[k]);
    }
    for (int c = 0; c < 2 * K; ++c)
        for (int q = 0; q < TKDV_MIX_R; ++q) {
            if (!std::isfinite(m.V[c][q])) return TKDV_E_ARG;
            V[c * TKDV_MIX_R + q] = m.V[c][q];
        }
    double g[2][2] = {{1.0, 0.0}, {0.0, 1.0}};
    for (int c = 0; c < 2 * K; ++c)
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) g[p][q] += V[c * 2 + p] * a[c] * V[c * 2 + q];
    const double det = g[0][0] * g[1][1] - g[0][1] * g[1][0];
    if (!(det > 0.0) || !std::isfinite(det)) return TKDV_E_ARG;
    std::memcpy(G, g, sizeof(G));
    Ginv[0][0] = g[1][1] / det;
    Ginv[1][1] = g[0][0] / det;
    Ginv[0][1] = -g[0][1] / det;
    Ginv[1][0] = -g[1][0] / det;
    logdetL0 = ldD + std::log(det);
    cs.assign((size_t)TKDV_MIX_S * K, 0.0);
    sn.assign(cs.size(), 0.0);
    for (int j = 0; j < TKDV_MIX_S; ++j)
        for (int k = 1; k <= K; ++k) {
            // angle k * 2 pi j / S reduced exactly
            const long r = ((long)k * j) % TKDV_MIX_S;
            const double ang = 2.0 * kPiH * (double)r / TKDV_MIX_S;
            cs[(size_t)j * K + k - 1] = std::cos(ang);
            sn[(size_t)j * K + k - 1] = std::sin(ang);
        }
    return TKDV_OK;
}

void MixHost::rot_inv(int j, const double *x, double *w) const
{
    for (int k = 0; k < K; ++k) {
        const double c = cs[(size_t)j * K + k], s = sn[(size_t)j * K + k];
        // shift by -phi: cos unchanged, sin negated
        w[k] = x[k] * c - x[K + k] * s;
        w[K + k] = x[K + k] * c + x[k] * s;
    }
}

void MixHost::rot(int j, const double *w, double *x) const
{
    for (int k = 0; k < K; ++k) {
        const double c = cs[(size_t)j * K + k], s = sn[(size_t)j * K + k];
        x[k] = w[k] * c + w[K + k] * s;
        x[K + k] = w[K + k] * c - w[k] * s;
    }
}

void MixHost::log_q(const double *x, double *lnet, double *lmix, double *grad) const
{
    const int n = 2 * K;
    std::vector<double> w(n), e(n), lj(TKDV_MIX_S), qf(TKDV_MIX_S);
    std::vector<double> Ae;  // per component A e_j, kept for the gradient
    if (grad) Ae.assign((size_t)TKDV_MIX_S * n, 0.0);
    double mx = -INFINITY;
    for (int j = 0; j < TKDV_MIX_S; ++j) {
        rot_inv(j, x, w.data());
        double y0 = 0.0, y1 = 0.0;
        for (int c = 0; c < n; ++c) {
            y0 += V[c * 2] * a[c] * w[c];
            y1 += V[c * 2 + 1] * a[c] * w[c];
        }
        const double g0 = Ginv[0][0] * y0 + Ginv[0][1] * y1, g1 = Ginv[1][0] * y0 + Ginv[1][1] * y1;
        double q = g0 * g0 + g1 * g1;
        for (int c = 0; c < n; ++c) {
            e[c] = w[c] - (V[c * 2] * g0 + V[c * 2 + 1] * g1);
            q += a[c] * e[c] * e[c];
            if (grad) Ae[(size_t)j * n + c] = a[c] * e[c];
        }
        qf[j] = q;
        lj[j] = -0.5 * logdetL0 - K * std::log(q);
        mx = std::max(mx, lj[j]);
    }
    double se = 0.0;
    for (int j = 0; j < TKDV_MIX_S; ++j) se += std::exp(lj[j] - mx);
    const double ln = mx + std::log(se) - std::log((double)TKDV_MIX_S);
    double t = 0.0;
    for (int k = 1; k <= K; ++k) t += (double)k * k * (x[k - 1] * x[k - 1] + x[K + k - 1] * x[K + k - 1]);
    const double gc = alpha * beta_p / ((double)K * K * K);
    const double lg = lng - K * std::log1p(gc * t);
    const double A1 = log_eps + lg, B1 = log_1m_eps + ln;
    const double hi = std::max(A1, B1);
    const double lm = hi + std::log(std::exp(A1 - hi) + std::exp(B1 - hi));
    if (lnet) *lnet = ln;
    if (lmix) *lmix = lm;
    if (grad) {
        // d log q_mix = wg d lg + wn d lnet; d lnet = sum_j pi_j d l_j,
        // d l_j = -K/qf_j * R_j (2 A e_j); d lg = -K gc/(1 + gc t) * 2 k^2 x
        const double wg = std::exp(A1 - lm), wn = std::exp(B1 - lm);
        std::vector<double> tmp(n), r(n);
        std::fill(grad, grad + n, 0.0);
        for (int j = 0; j < TKDV_MIX_S; ++j) {
            const double pij = std::exp(lj[j] - mx) / se;
            const double cj = wn * pij * (-K / qf[j]) * 2.0;
            rot(j, &Ae[(size_t)j * n], r.data());
            for (int c = 0; c < n; ++c) grad[c] += cj * r[c];
        }
        const double dg = wg * (-K * gc / (1.0 + gc * t));
        for (int c = 0; c < n; ++c) {
            const int k = c % K + 1;
            grad[c] += dg * 2.0 * k * k * x[c];
        }
    }
}

double MixHost::kappa() const
{
    const double tr = G[0][0] + G[1][1], det = G[0][0] * G[1][1] - G[0][1] * G[1][0];
    const double disc = std::sqrt(std::max(0.0, tr * tr / 4.0 - det));
    return tr / 2.0 + disc;
}

template <int K>
static void mix_tables(const MixHost &mh, std::vector<uint8_t> &tab)
{
    const int nb = mix_ytab_bf16_bytes<K>(), nf = mix_ytab_f32_bytes<K>(), nr = mix_rv_bytes<K>();
    tab.assign((size_t)mix_point_bytes<K>(), 0);
    uint16_t *yh = reinterpret_cast<uint16_t *>(tab.data());
    uint16_t *yl = reinterpret_cast<uint16_t *>(tab.data() + nb);
    float *yf = reinterpret_cast<float *>(tab.data() + 2 * nb);
    float *rv = reinterpret_cast<float *>(tab.data() + 2 * nb + nf);
    (void)nr;
    // RV[j][c][q] = (R_j V_q)_c
    std::vector<double> R((size_t)TKDV_MIX_S * 2 * K * 2);
    for (int j = 0; j < TKDV_MIX_S; ++j)
        for (int q = 0; q < 2; ++q) {
            std::vector<double> v(2 * K), r(2 * K);
            for (int c = 0; c < 2 * K; ++c) v[c] = mh.V[c * 2 + q];
            mh.rot(j, v.data(), r.data());
            for (int c = 0; c < 2 * K; ++c) R[((size_t)j * 2 * K + c) * 2 + q] = r[c];
        }
    // C: upper Cholesky factor of G^-1 = (I + V^T D^-1 V)^-1 = C^T C; the
    // tables hold A R_j V C^T, so the products give z_j = C y_j directly
    const double c00 = std::sqrt(mh.Ginv[0][0]), c01 = mh.Ginv[0][1] / c00;
    const double c11 = std::sqrt(std::max(0.0, mh.Ginv[1][1] - c01 * c01));
    const double C[2][2] = {{c00, c01}, {0.0, c11}};
    auto B = [&](int q, int j, int c) {
        const double *r = &R[((size_t)j * 2 * K + c) * 2];
        return mh.a[c] * (C[q][0] * r[0] + C[q][1] * r[1]);
    };
    for (int t = 0; t < 2; ++t)
        for (int s = 0; s < K / 8; ++s)
            for (int l = 0; l < 64; ++l)
                for (int e = 0; e < 8; ++e) {
                    const int j = l % 32, c = (l / 32) * K + 8 * s + e;
                    const double v = B(t, j, c);
                    const uint16_t h = bf16_bits((float)v);
                    const size_t idx = (((size_t)t * (K / 8) + s) * 64 + l) * 8 + e;
                    yh[idx] = h;
                    yl[idx] = bf16_bits((float)(v - (double)bf16_value(h)));
                }
    for (int t = 0; t < 2; ++t)
        for (int q = 0; q < K / 4; ++q)
            for (int l = 0; l < 64; ++l)
                for (int e = 0; e < 4; ++e) {
                    const int j = l % 32, c = (l / 32) * K + 4 * q + e;
                    yf[(((size_t)t * (K / 4) + q) * 64 + l) * 4 + e] = (float)B(t, j, c);
                }
    for (int j = 0; j < TKDV_MIX_S; ++j)
        for (int h = 0; h < 2; ++h)
            for (int k = 0; k < K; ++k)
                for (int q = 0; q < 2; ++q)
                    rv[(size_t)(2 * j + h) * (2 * K + 2) + 2 * k + q] =
                        (float)R[((size_t)j * 2 * K + h * K + k) * 2 + q];
}

void mix_device_data(const MixHost &mh, DevMix &d, std::vector<uint8_t> &tab)
{
    std::memset(&d, 0, sizeof(d));
    const int K = mh.K;
    for (int k = 0; k < K; ++k) {
        d.sqd[k] = (float)mh.sqd[k];
        d.a[k] = (float)mh.a[k];
        d.sqd64[k] = mh.sqd[k];
        d.a64[k] = mh.a[k];
    }
    for (int c = 0; c < 2 * K; ++c)
        for (int q = 0; q < 2; ++q) d.V64[c][q] = mh.V[c * 2 + q];
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q) d.gi64[p][q] = mh.Ginv[p][q];
    d.c_net = (float)(mh.log_1m_eps - 0.5 * mh.logdetL0 - std::log((double)TKDV_MIX_S));
    d.c_g = (float)(mh.log_eps + mh.lng);
    d.E = (uint32_t)mh.E;
    d.B = (uint32_t)(((1ull << 32) - mh.E) / TKDV_MIX_S);
    d.invB = (float)(1.0 / (double)d.B);
    for (int m = 0; m < TKDV_MIX_S; ++m) {
        d.cs64[m] = std::cos(2.0 * kPiH * m / TKDV_MIX_S);
        d.sn64[m] = std::sin(2.0 * kPiH * m / TKDV_MIX_S);
    }
    d.logdetL0 = mh.logdetL0;
    d.lng = mh.lng;
    d.log_eps = mh.log_eps;
    d.log_1m_eps = mh.log_1m_eps;
    switch (K) {
    case 8: mix_tables<8>(mh, tab); break;
    case 16: mix_tables<16>(mh, tab); break;
    case 32: mix_tables<32>(mh, tab); break;
    case 64: mix_tables<64>(mh, tab); break;
    default: tab.clear();
    }
}

double mix_window_extra(const MixHost &mh, int precision)
{
    const int K = mh.K;
    const double eps_x = 1e-5;  // bound on |x^_fast - x^_exact|_2 of the draw
    double eps_p;               // relative error of the y products (per sum of |terms|)
    switch (precision) {
    case TKDV_FP32: eps_p = 2.0 * K * 0x1p-23; break;
    case TKDV_BF16: eps_p = 1.01 * 0x1p-8 + 2.0 * K * 0x1p-23; break;
    default: eps_p = 3.02 * 0x1p-18 + 2.0 * K * 0x1p-23; break;
    }
    double dmin = INFINITY, dmax = 0.0, vf2 = 0.0, avf2 = 0.0;
    for (int k = 0; k < K; ++k) {
        dmin = std::min(dmin, 1.0 / mh.a[k]);
        dmax = std::max(dmax, 1.0 / mh.a[k]);
    }
    for (int c = 0; c < 2 * K; ++c) {
        const double n2 = mh.V[c * 2] * mh.V[c * 2] + mh.V[c * 2 + 1] * mh.V[c * 2 + 1];
        vf2 += n2;
        avf2 += mh.a[c] * mh.a[c] * n2;
    }
    const double kap = mh.kappa();
    const double amin = 1.0 / dmax;
    const double cond = (dmax + vf2) / dmin;
    // (a) x^ error: |d ln qf_j| <= 2 |dx| sqrt(cond L0)
    const double e_in = K * 2.0 * eps_x * std::sqrt(cond);
    // (b) y products: |d qf|/qf <= 2 kappa eps_p |A V|_F / sqrt(a_min); the
    //     products form z = C y with C^T C = G^-1, and |A V C^T|_F <= |A V|_F
    //     because |C|_2^2 = |G^-1|_2 <= 1 (G = I + V^T D^-1 V >= I)
    const double e_y = K * 2.0 * kap * eps_p * std::sqrt(avf2) / std::sqrt(amin);
    // (c) FP32 rounding of Q, the 2x2 form and r_j = 1 - quad/Q, relative to r_j >= 1/kappa
    const double e_r = K * kap * (2.0 * K + 10.0) * 0x1p-24;
    // (d) hardware log2/exp2 of the terms and of the sums
    const double e_tr = (4.0 * K + 40.0) * 0x1p-22;
    // (e) rounding of the combination, by the magnitudes of its terms
    const double gc = mh.alpha * mh.beta_p / ((double)K * K * K);
    const double magN = std::fabs(mh.log_1m_eps - 0.5 * mh.logdetL0) + std::log((double)TKDV_MIX_S) +
                        K * (std::fabs(std::log(amin)) + std::fabs(std::log(1.0 / dmin)) + std::log(kap));
    const double magG = std::fabs(mh.log_eps + mh.lng) + K * std::log1p(gc * K * K);
    const double e_c = 16.0 * 0x1p-24 * (magN + magG + 30.0);
    return e_in + e_y + e_r + e_tr + e_c;
}

// log f - log q_mix on the sphere: value and tangent gradient.
struct MixObjective {
    GradEval fe;  // log f (uniform-proposal objective: no proposal term)
    const MixHost &mh;
    MixObjective(const tkdv_point &pt, const MixHost &m)
        : fe(Objective{pt.K, pt.E0, pt.beta_p, pt.c32, 1.0, TKDV_PROP_UNIFORM}), mh(m) {}
    double operator()(const std::vector<double> &x, std::vector<double> &g) const
    {
        const double lf = fe(x, g);  // tangent gradient of log f
        const int n = (int)x.size();
        std::vector<double> gq(n);
        double lm;
        mh.log_q(x.data(), nullptr, &lm, gq.data());
        double gx = 0.0;
        for (int c = 0; c < n; ++c) gx += gq[c] * x[c];
        for (int c = 0; c < n; ++c) g[c] -= gq[c] - gx * x[c];
        return lf - lm;
    }
};

}  // namespace tkdv

using namespace tkdv;

extern "C" tkdv_status tkdv_mixture_log_q(const tkdv_point *pt, const tkdv_plan *sp, const tkdv_mixture *mix,
                                          const double *xhat, int32_t n, double *lnet, double *lmix)
{
    if (!pt || !sp || !mix || (n > 0 && !xhat)) return TKDV_E_ARG;
    MixHost mh;
    const int st = mh.init(*pt, *sp, *mix);
    if (st != TKDV_OK) return (tkdv_status)st;
    for (int32_t i = 0; i < n; ++i)
        mh.log_q(xhat + (size_t)i * 2 * pt->K, lnet ? lnet + i : nullptr, lmix ? lmix + i : nullptr, nullptr);
    return TKDV_OK;
}

extern "C" tkdv_status tkdv_plan_mixture(const tkdv_point *pt, const tkdv_plan *sp, const tkdv_mixture *mix,
                                         const double *starts, int32_t n_starts, double margin, tkdv_plan *out,
                                         double *argmax)
{
    if (!pt || !sp || !mix || !out || n_starts < 0 || (n_starts > 0 && !starts) || !(margin >= 0.0))
        return TKDV_E_ARG;
    if (sp->proposal != TKDV_PROP_SIGMA) return TKDV_E_ARG;
    MixHost mh;
    int st = mh.init(*pt, *sp, *mix);
    if (st != TKDV_OK) return (tkdv_status)st;
    const int K = pt->K, n = 2 * K;
    MixObjective obj(*pt, mh);
    std::vector<std::vector<double>> S;
    // zero-mean Dirichlet kernel and its S shifts, the single-mode state
    {
        std::vector<double> d(n, 0.0), r(n);
        for (int k = 0; k < K; ++k) d[k] = 1.0 / std::sqrt((double)K);
        for (int j = 0; j < TKDV_MIX_S; j += 4) {
            mh.rot(j, d.data(), r.data());
            S.push_back(r);
        }
        std::vector<double> e1(n, 0.0);
        e1[0] = 1.0;
        S.push_back(e1);
    }
    // the Sigma maximiser (from the Dirichlet kernel)
    {
        Objective os{K, pt->E0, pt->beta_p, pt->c32, sp->alpha_star, TKDV_PROP_SIGMA};
        GradEval gs(os);
        std::vector<double> d(n, 0.0);
        for (int k = 0; k < K; ++k) d[k] = 1.0 / std::sqrt((double)K);
        long ev = 0;
        bfgs_polish(gs, d, &ev);
        S.push_back(d);
    }
    for (int32_t s = 0; s < n_starts; ++s) {
        std::vector<double> v(starts + (size_t)s * n, starts + (size_t)(s + 1) * n);
        double r = 0.0;
        for (double z : v) r += z * z;
        if (!(r > 0.0) || !std::isfinite(r)) return TKDV_E_ARG;
        for (double &z : v) z /= std::sqrt(r);
        S.push_back(v);
    }
    {
        uint64_t s = 0x9E3779B97F4A7C15ull ^ (uint64_t)K;
        for (int q = 0; q < 4; ++q) {
            std::vector<double> v(n);
            double r = 0.0;
            for (int c = 0; c < n; ++c) {
                s += 0x9E3779B97F4A7C15ull;
                uint64_t z = (s ^ (s >> 30)) * 0xBF58476D1CE4E5B9ull;
                z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
                z ^= z >> 31;
                v[c] = ((double)(z >> 11) * 0x1p-53) - 0.5;
                r += v[c] * v[c];
            }
            for (double &z : v) z /= std::sqrt(r);
            S.push_back(v);
        }
    }
    std::vector<double> vals(S.size());
    std::vector<long> evs(S.size(), 0);
    {
        const size_t nt = std::min<size_t>(S.size(), std::max(1u, std::thread::hardware_concurrency()));
        std::vector<std::thread> th;
        for (size_t w = 0; w < nt; ++w)
            th.emplace_back([&, w] {
                for (size_t s = w; s < S.size(); s += nt) vals[s] = bfgs_polish(obj, S[s], &evs[s]);
            });
        for (auto &t : th) t.join();
    }
    size_t best = 0;
    long total = 0;
    for (size_t s = 0; s < S.size(); ++s) {
        if (vals[s] > vals[best]) best = s;
        total += evs[s];
    }
    const double cap = sp->log_M - sp->log_norm_g - mh.log_eps;
    double lm = vals[best] + std::log1p(margin);
    *out = *sp;
    out->proposal = TKDV_PROP_MIXTURE;
    out->log_M = std::min(lm, cap);
    out->M_source = lm > cap ? 3 : 1;
    out->n_optimiser_evals = (int32_t)std::min<long>(total, INT32_MAX);
    if (argmax) std::memcpy(argmax, S[best].data(), sizeof(double) * n);
    return TKDV_OK;
}
