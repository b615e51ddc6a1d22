// Host precompute of the rejection algorithm (step 1 of Sec. IV.B) in FP64:
//   * alpha* = root of F(alpha) = 1 - (alpha/K) sum_k 1/(1 + alpha beta' k^2/K^3)
//     (Sec. III.A) by Brent's method on a bracket found by doubling;
//   * the proposal variances s_k^2 = 1/(1 + alpha* beta' k^2/K^3);
//   * log M, M = sup over the sphere of the unnormalised ratio f/g (Sec. IV.A):
//     closed form when C3/C2 = 0, otherwise adaptive Nelder-Mead started at
//     the zero-mean Dirichlet kernel (the paper's initial guess, Sec. IV.A),
//     at the single-mode state and at seeded random directions; each run is
//     polished by BFGS ascent on the sphere with the analytic gradient and
//     restarted from its incumbent until a restart gains nothing.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

#include "tkdv_host_math.h"
#include "tkdv_plan.h"

namespace tkdv {

static const double kPi = 3.14159265358979323846;

double plan_F(int K, double beta_p, double alpha)
{
    const double K3 = (double)K * K * K;
    double s = 0.0;
    for (int k = 1; k <= K; ++k) s += 1.0 / (1.0 + alpha * beta_p * (double)k * k / K3);
    return 1.0 - alpha * s / K;
}

bool plan_alpha_root_exists(int K, double beta_p)
{
    double s = 0.0;
    for (int k = 1; k <= K; ++k) s += 1.0 / ((double)k * k);
    return beta_p >= 0.0 && beta_p < (double)K * K * s;
}

// Brent's method (inverse quadratic interpolation / secant / bisection) for a
// root of a continuous function bracketed by [a, b] with f(a) f(b) <= 0.
template <class Fn>
static double brent_root(Fn f, double a, double b, double fa, double fb)
{
    double c = a, fc = fa, d = b - a, e = d;
    for (int it = 0; it < 300; ++it) {
        if ((fb > 0 && fc > 0) || (fb < 0 && fc < 0)) { c = a; fc = fa; d = e = b - a; }
        if (std::fabs(fc) < std::fabs(fb)) { a = b; b = c; c = a; fa = fb; fb = fc; fc = fa; }
        const double tol = 2.0 * 2.220446049250313e-16 * std::fabs(b) + 1e-300;
        const double m = 0.5 * (c - b);
        if (std::fabs(m) <= tol || fb == 0.0) return b;
        if (std::fabs(e) >= tol && std::fabs(fa) > std::fabs(fb)) {
            double s = fb / fa, p, q;
            if (a == c) {
                p = 2.0 * m * s;
                q = 1.0 - s;
            } else {
                double qq = fa / fc, r = fb / fc;
                p = s * (2.0 * m * qq * (qq - r) - (b - a) * (r - 1.0));
                q = (qq - 1.0) * (r - 1.0) * (s - 1.0);
            }
            if (p > 0) q = -q; else p = -p;
            if (2.0 * p < std::min(3.0 * m * q - std::fabs(tol * q), std::fabs(e * q))) {
                e = d;
                d = p / q;
            } else {
                d = m;
                e = m;
            }
        } else {
            d = m;
            e = m;
        }
        a = b;
        fa = fb;
        b += (std::fabs(d) > tol) ? d : (m > 0 ? tol : -tol);
        fb = f(b);
    }
    return b;
}

int plan_alpha_star(int K, double beta_p, double *out)
{
    if (!(beta_p >= 0.0) || !std::isfinite(beta_p)) return TKDV_E_ARG;
    if (beta_p == 0.0) { *out = 1.0; return TKDV_OK; }
    if (!plan_alpha_root_exists(K, beta_p)) return TKDV_E_NO_ALPHA_ROOT;
    double hi = 1.0;
    double fhi = plan_F(K, beta_p, hi);
    while (fhi > 0.0) {
        hi *= 2.0;
        if (hi > 1e300) return TKDV_E_NO_ALPHA_ROOT;
        fhi = plan_F(K, beta_p, hi);
    }
    auto f = [&](double a) { return plan_F(K, beta_p, a); };
    *out = brent_root(f, 0.0, hi, 1.0, fhi);
    return TKDV_OK;
}

// Adaptive Nelder-Mead (Gao & Han 2012 coefficients) maximising obj from y0.
static double nelder_mead_max(const Objective &obj, std::vector<double> &y, long max_evals,
                              long *evals)
{
    const int n = 2 * obj.K;
    const double rho = 1.0, chi = 1.0 + 2.0 / n, psi = 0.75 - 1.0 / (2.0 * n), sig = 1.0 - 1.0 / n;
    std::vector<std::vector<double>> S(n + 1, y);
    std::vector<double> f(n + 1);
    for (int i = 0; i < n; ++i) {
        double &v = S[i + 1][i];
        v = (v != 0.0) ? 1.05 * v : 0.00025;
    }
    // minimise -obj
    for (int i = 0; i <= n; ++i) f[i] = -obj(S[i].data());
    long ev = n + 1;
    std::vector<int> order(n + 1);
    std::vector<double> xb(n), xr(n), xe(n), xc(n);
    while (ev < max_evals) {
        for (int i = 0; i <= n; ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](int a, int b) { return f[a] < f[b]; });
        {
            std::vector<std::vector<double>> S2(n + 1);
            std::vector<double> f2(n + 1);
            for (int i = 0; i <= n; ++i) { S2[i].swap(S[order[i]]); f2[i] = f[order[i]]; }
            S.swap(S2);
            f.swap(f2);
        }
        double fspread = 0.0, xspread = 0.0;
        for (int i = 1; i <= n; ++i) {
            fspread = std::max(fspread, std::fabs(f[i] - f[0]));
            for (int m = 0; m < n; ++m) xspread = std::max(xspread, std::fabs(S[i][m] - S[0][m]));
        }
        if (fspread <= 1e-13 && xspread <= 1e-6) break;
        std::fill(xb.begin(), xb.end(), 0.0);
        for (int i = 0; i < n; ++i)
            for (int m = 0; m < n; ++m) xb[m] += S[i][m];
        for (int m = 0; m < n; ++m) xb[m] /= n;
        for (int m = 0; m < n; ++m) xr[m] = (1 + rho) * xb[m] - rho * S[n][m];
        const double fr = -obj(xr.data());
        ++ev;
        bool shrink = false;
        if (fr < f[0]) {
            for (int m = 0; m < n; ++m) xe[m] = (1 + rho * chi) * xb[m] - rho * chi * S[n][m];
            const double fe = -obj(xe.data());
            ++ev;
            if (fe < fr) { S[n] = xe; f[n] = fe; } else { S[n] = xr; f[n] = fr; }
        } else if (fr < f[n - 1]) {
            S[n] = xr;
            f[n] = fr;
        } else if (fr < f[n]) {
            for (int m = 0; m < n; ++m) xc[m] = (1 + psi * rho) * xb[m] - psi * rho * S[n][m];
            const double fc = -obj(xc.data());
            ++ev;
            if (fc <= fr) { S[n] = xc; f[n] = fc; } else shrink = true;
        } else {
            for (int m = 0; m < n; ++m) xc[m] = (1 - psi) * xb[m] + psi * S[n][m];
            const double fc = -obj(xc.data());
            ++ev;
            if (fc < f[n]) { S[n] = xc; f[n] = fc; } else shrink = true;
        }
        if (shrink) {
            for (int i = 1; i <= n; ++i) {
                for (int m = 0; m < n; ++m) S[i][m] = S[0][m] + sig * (S[i][m] - S[0][m]);
                f[i] = -obj(S[i].data());
                ++ev;
            }
        }
    }
    int best = 0;
    for (int i = 1; i <= n; ++i) if (f[i] < f[best]) best = i;
    y = S[best];
    double r = 0.0;
    for (double v : y) r += v * v;
    r = std::sqrt(r);
    for (double &v : y) v /= r;
    *evals += ev;
    return -f[best];
}

static double maximise_from(const Objective &obj, std::vector<double> y, long *evals)
{
    double r = 0.0;
    for (double v : y) r += v * v;
    r = std::sqrt(r);
    for (double &v : y) v /= r;
    GradEval ge(obj);
    double best = obj(y.data());
    for (int restart = 0; restart < 6; ++restart) {
        std::vector<double> z = y;
        double v = nelder_mead_max(obj, z, 20000 + 400L * obj.K, evals);
        bfgs_polish(ge, z, evals);
        v = obj(z.data());
        const bool improved = v > best + 1e-14;
        if (v > best) { best = v; y = z; }
        if (!improved) break;
    }
    return best;
}

static uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int plan_base_host(const tkdv_point *pt, int proposal, tkdv_plan *out)
{
    if (!pt || !out) return TKDV_E_ARG;
    const int K = pt->K;
    if (K < 1 || K > TKDV_KMAX) return TKDV_E_ARG;
    if (!std::isfinite(pt->E0) || !(pt->E0 > 0.0)) return TKDV_E_ARG;
    if (!std::isfinite(pt->beta_p) || pt->beta_p < 0.0) return TKDV_E_ARG;
    if (!std::isfinite(pt->c32)) return TKDV_E_ARG;
    if (proposal != TKDV_PROP_UNIFORM && proposal != TKDV_PROP_SIGMA) return TKDV_E_ARG;
    std::memset(out, 0, sizeof(*out));
    out->N = 4 * K;
    out->proposal = proposal;
    double alpha = 1.0;
    if (proposal == TKDV_PROP_SIGMA) {
        const int st = plan_alpha_star(K, pt->beta_p, &alpha);
        if (st != TKDV_OK) return st;
    }
    out->alpha_star = alpha;
    const double K3 = (double)K * K * K;
    for (int k = 1; k <= TKDV_KMAX; ++k) {
        out->sigma2[k - 1] = (proposal == TKDV_PROP_SIGMA && k <= K)
                                 ? 1.0 / (1.0 + alpha * pt->beta_p * (double)k * k / K3)
                                 : 1.0;
        if (proposal == TKDV_PROP_SIGMA && k <= K)
            out->log_norm_g += std::log1p(alpha * pt->beta_p * (double)k * k / K3);
    }
    if (pt->c32 == 0.0) {
        // f/g = h(t); log h concave in t, stationary at t* = K^3 (alpha-1)/(alpha beta'),
        // t ranges over [1, K^2] on the sphere.  Uniform: f largest at t = 1.
        out->M_source = 0;
        if (proposal == TKDV_PROP_UNIFORM) {
            out->log_M = -pt->beta_p / ((double)K * K);
        } else if (pt->beta_p == 0.0) {
            out->log_M = 0.0;
        } else {
            double ts = K3 * (alpha - 1.0) / (alpha * pt->beta_p);
            ts = std::min(std::max(ts, 1.0), (double)K * K);
            out->log_M = -pt->beta_p * ts / ((double)K * K) + K * std::log1p(alpha * pt->beta_p * ts / K3);
        }
        return TKDV_OK;
    }
    out->M_source = -1;
    return TKDV_OK;
}

int plan_point_host(const tkdv_point *pt, int proposal, int n_random, tkdv_plan *out)
{
    const int st = plan_base_host(pt, proposal, out);
    if (st != TKDV_OK || out->M_source == 0) return st;
    const int K = pt->K;
    const double alpha = out->alpha_star;
    Objective obj{K, pt->E0, pt->beta_p, pt->c32, alpha, proposal};
    std::vector<std::vector<double>> starts;
    {
        std::vector<double> y(2 * K, 0.0);
        for (int k = 0; k < K; ++k) y[k] = 1.0;  // zero-mean Dirichlet kernel
        starts.push_back(y);
        std::vector<double> e1(2 * K, 0.0);
        e1[0] = 1.0;  // all energy in mode 1
        starts.push_back(e1);
        uint64_t s = 0x5EED0F7D4C0FFEEull ^ (uint64_t)K;
        for (int r = 0; r < n_random; ++r) {
            std::vector<double> g(2 * K);
            for (int m = 0; m < 2 * K; m += 2) {
                const double u1 = ((splitmix64(s) >> 11) + 0.5) * 0x1p-53;
                const double u2 = ((splitmix64(s) >> 11) + 0.5) * 0x1p-53;
                const double rr = std::sqrt(-2.0 * std::log(u1));
                g[m] = rr * std::cos(2 * kPi * u2);
                if (m + 1 < 2 * K) g[m + 1] = rr * std::sin(2 * kPi * u2);
            }
            starts.push_back(g);
        }
    }
    std::vector<double> vals(starts.size());
    std::vector<long> evs(starts.size(), 0);
    {
        std::vector<std::thread> th;
        for (size_t s = 0; s < starts.size(); ++s)
            th.emplace_back([&, s] { vals[s] = maximise_from(obj, starts[s], &evs[s]); });
        for (auto &t : th) t.join();
    }
    double best = -INFINITY;
    long total = 0;
    for (size_t s = 0; s < starts.size(); ++s) {
        best = std::max(best, vals[s]);
        total += evs[s];
    }
    out->log_M = best;
    out->M_source = 1;
    out->n_optimiser_evals = (int32_t)std::min<long>(total, INT32_MAX);
    return TKDV_OK;
}

double plan_log_ratio(const tkdv_point *pt, const tkdv_plan *pl, const double *xhat)
{
    Objective obj{pt->K, pt->E0, pt->beta_p, pt->c32, pl->alpha_star, pl->proposal};
    return obj(xhat);
}

}  // namespace tkdv
