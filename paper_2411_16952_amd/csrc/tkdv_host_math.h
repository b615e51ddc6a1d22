// Host FP64 helpers shared by the plan and the mixture search: the log of the
// unnormalised target/proposal ratio on the sphere, its Riemannian gradient,
// and BFGS ascent on the sphere.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/tkdv.h"

namespace tkdv {

static const double kPiH = 3.14159265358979323846;

// Round to bfloat16 with round-to-nearest-even; returns the bits.
inline uint16_t bf16_bits(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}
inline float bf16_value(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// ---------------------------------------------------------------------------
// The objective: log of the unnormalised ratio at y/|y|.
//   log f/g = -beta'/(E0 K^2) (H2 - c H3) + K log(1 + alpha beta' t/K^3)  (Sigma)
//   log f   = -beta'/(E0 K^2) (H2 - c H3)                                (uniform)
// H3 by the double sum over triads k + (n - k) = n (Sec. IV.A).
// ---------------------------------------------------------------------------
struct Objective {
    int K;
    double E0, beta_p, c32, alpha;
    int proposal;

    double operator()(const double *y) const
    {
        double r2 = 0.0;
        for (int m = 0; m < 2 * K; ++m) r2 += y[m] * y[m];
        const double inv = 1.0 / std::sqrt(r2);
        double re[TKDV_KMAX + 1], im[TKDV_KMAX + 1];
        double t = 0.0;
        for (int k = 1; k <= K; ++k) {
            const double a = y[k - 1] * inv, b = y[K + k - 1] * inv;
            re[k] = a;
            im[k] = -b;
            t += (double)k * k * (a * a + b * b);
        }
        // sum_n Re(conj(v_n) sum_{k<n} v_k v_{n-k}), v_k = x^_k - i x^_{K+k}
        double tri = 0.0;
        for (int n = 2; n <= K; ++n) {
            double sr = 0.0, si = 0.0;
            for (int k = 1; k < n; ++k) {
                sr += re[k] * re[n - k] - im[k] * im[n - k];
                si += re[k] * im[n - k] + im[k] * re[n - k];
            }
            tri += re[n] * sr + im[n] * si;
        }
        const double H3 = 2.0 * kPiH * std::pow(E0 / (2.0 * kPiH), 1.5) * tri;
        const double H2 = E0 * t;
        double v = -beta_p / (E0 * (double)K * K) * (H2 - c32 * H3);
        if (proposal == TKDV_PROP_SIGMA) v += K * std::log1p(alpha * beta_p * t / ((double)K * K * K));
        return v;
    }
};

// Value and Riemannian gradient of the objective at x^ on the sphere.  The
// gradient of H3 uses the exact grid quadrature (N = 4K >= 3K + 1, so
// u^2 cos k xi is integrated exactly): dH3/dx^_m = (pi amp/N) sum_j u_j^2 Phi_mj.
struct GradEval {
    const Objective obj;
    int N;
    std::vector<double> cs, sn;  // [N][K]
    explicit GradEval(const Objective &o) : obj(o), N(4 * o.K), cs((size_t)4 * o.K * o.K), sn(cs.size())
    {
        const int K = o.K;
        for (int j = 0; j < N; ++j)
            for (int k = 1; k <= K; ++k) {
                const long r = ((long)k * j) % N;
                const double ang = 2.0 * kPiH * (double)r / N, sg = (k & 1) ? -1.0 : 1.0;
                cs[(size_t)j * K + k - 1] = sg * std::cos(ang);
                sn[(size_t)j * K + k - 1] = sg * std::sin(ang);
            }
    }
    double operator()(const std::vector<double> &x, std::vector<double> &g) const
    {
        const int K = obj.K;
        const double amp = std::sqrt(2.0 * obj.E0 / kPiH);
        double t = 0.0;
        for (int k = 1; k <= K; ++k) t += (double)k * k * (x[k - 1] * x[k - 1] + x[K + k - 1] * x[K + k - 1]);
        std::vector<double> dh3(2 * K, 0.0);
        double h3 = 0.0;
        for (int j = 0; j < N; ++j) {
            double u = 0.0;
            for (int k = 0; k < K; ++k) u += x[k] * cs[(size_t)j * K + k] + x[K + k] * sn[(size_t)j * K + k];
            u *= amp;
            h3 += u * u * u;
            const double w = u * u;
            for (int k = 0; k < K; ++k) {
                dh3[k] += w * cs[(size_t)j * K + k];
                dh3[K + k] += w * sn[(size_t)j * K + k];
            }
        }
        h3 *= kPiH / (3.0 * N);
        const double cH = obj.beta_p * obj.c32 / (obj.E0 * (double)K * K);
        double dt = -obj.beta_p / ((double)K * K);
        double val = -obj.beta_p / ((double)K * K) * t + cH * h3;
        if (obj.proposal == TKDV_PROP_SIGMA) {
            const double a = obj.alpha * obj.beta_p / ((double)K * K * K);
            val += K * std::log1p(a * t);
            dt += K * a / (1.0 + a * t);
        }
        g.assign(2 * K, 0.0);
        for (int m = 0; m < 2 * K; ++m) {
            const int k = m % K + 1;
            g[m] = dt * 2.0 * k * k * x[m] + cH * (kPiH * amp / N) * dh3[m];
        }
        double gx = 0.0;
        for (int m = 0; m < 2 * K; ++m) gx += g[m] * x[m];
        for (int m = 0; m < 2 * K; ++m) g[m] -= gx * x[m];  // tangent component
        return val;
    }
};

// BFGS ascent on the sphere (retraction by normalisation, Armijo backtracking).
template <class F>
inline double bfgs_polish(const F &ge, std::vector<double> &x, long *evals)
{
    const int n = (int)x.size();
    std::vector<double> g(n), g2(n), x2(n), d(n), s(n), yv(n), Hy(n);
    std::vector<double> H((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) H[(size_t)i * n + i] = 1.0;
    double f = ge(x, g);
    ++*evals;
    for (int it = 0; it < 2000; ++it) {
        double gn = 0.0;
        for (double v : g) gn += v * v;
        if (std::sqrt(gn) < 1e-13) break;
        for (int i = 0; i < n; ++i) {  // ascent direction H g
            double acc = 0.0;
            for (int j = 0; j < n; ++j) acc += H[(size_t)i * n + j] * g[j];
            d[i] = acc;
        }
        double slope = 0.0;
        for (int i = 0; i < n; ++i) slope += d[i] * g[i];
        if (!(slope > 0.0)) {  // reset to steepest ascent
            std::fill(H.begin(), H.end(), 0.0);
            for (int i = 0; i < n; ++i) H[(size_t)i * n + i] = 1.0;
            d = g;
            slope = gn;
        }
        double step = 1.0, f2 = f;
        bool ok = false;
        for (int ls = 0; ls < 60; ++ls) {
            double r = 0.0;
            for (int i = 0; i < n; ++i) { x2[i] = x[i] + step * d[i]; r += x2[i] * x2[i]; }
            r = std::sqrt(r);
            for (int i = 0; i < n; ++i) x2[i] /= r;
            f2 = ge(x2, g2);
            ++*evals;
            if (f2 >= f + 1e-4 * step * slope) { ok = true; break; }
            step *= 0.5;
        }
        if (!ok) break;
        double sy = 0.0;
        for (int i = 0; i < n; ++i) { s[i] = x2[i] - x[i]; yv[i] = g[i] - g2[i]; sy += s[i] * yv[i]; }
        const double gain = f2 - f;
        x = x2;
        g = g2;
        f = f2;
        if (sy > 1e-300) {  // BFGS update of the inverse Hessian of -f
            double yHy = 0.0;
            for (int i = 0; i < n; ++i) {
                double acc = 0.0;
                for (int j = 0; j < n; ++j) acc += H[(size_t)i * n + j] * yv[j];
                Hy[i] = acc;
                yHy += yv[i] * acc;
            }
            const double rho = 1.0 / sy;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j)
                    H[(size_t)i * n + j] += (1.0 + yHy * rho) * rho * s[i] * s[j] - rho * (Hy[i] * s[j] + s[i] * Hy[j]);
        }
        if (gain < 1e-16 * (1.0 + std::fabs(f)) && it > 5) break;
    }
    return f;
}


}  // namespace tkdv
