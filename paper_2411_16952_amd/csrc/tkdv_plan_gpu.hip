// Multi-start search for the rejection constant M = sup over the sphere of
// f/g (Sec. IV.A; step 1 of the algorithm of Sec. IV.B), one wavefront per
// (point, start), in FP64.
//
// Each wave maximises phi(x^) = log f(x^) - log g(x^) (the unnormalised ratio
// of tkdv_plan_point), or log f - log q_mix for the learned mixture (K <= 32),
// by L-BFGS ascent on the unit sphere: retraction by
// normalisation, the tangent gradient, Armijo backtracking, 8 curvature pairs
// kept in registers.  The value and the gradient come from the N = 4K grid:
//   u~_j = sum_k (-1)^k (x^_k cos(2 pi k j/N) + x^_{K+k} sin(2 pi k j/N)),
//   H3 = (pi/(3N)) amp^3 sum_j u~_j^3 (exact for N >= 3K + 1),
//   d/dx^_m sum_j u~_j^3 = 3 sum_j u~_j^2 Phi_mj,
// with one table of cos(2 pi r/N) in LDS (sin by a quarter-period offset).
// Lane l holds coordinates l + 64 c of x^ and the gradient (c < C: C = 2 for
// K <= 64, 4 for K = 128), and grid points l + 64 r.  Every branch taken on a wave-reduced quantity goes
// through readfirstlane, so all lanes of a wave follow one path.
#include "tkdv_device.h"
#include "tkdv_plan_gpu.h"

namespace tkdv {
namespace {

constexpr double kPiP = 3.14159265358979323846;

// Butterfly sum: every lane ends with the same bits (each stage adds the same
// two partial sums in both lanes of a pair).
__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ bool uniform(bool c) { return __builtin_amdgcn_readfirstlane((int)c) != 0; }

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// log q_mix of the mixture at the unit vector x (K <= 32: coordinate `lane`)
// and its ambient gradient for this lane's coordinate; t = sum_k k^2 s_k.
// The shifts' log-sum-exp runs online (rescaled when a larger term appears).
__device__ double mix_log_q(const PlanMix &M, int K, int lane, double x0, double t, double &dq)
{
    const int n2 = 2 * K;
    const bool act = lane < n2;
    const bool sinb = lane >= K;
    const int k = lane % K + 1;
    const int partner = act ? (sinb ? lane - K : lane + K) : lane;
    const double xp = __shfl(x0, partner, 64);
    const double am = act ? M.a[lane] : 0.0;
    const double v0 = act ? M.V[lane][0] : 0.0, v1 = act ? M.V[lane][1] : 0.0;
    double mx = -INFINITY, se = 0.0, G = 0.0;
    for (int j = 0; j < 32; ++j) {
        const int mi = (k * j) & 31;
        const double cs = M.cs[mi], sn = M.sn[mi];
        const double w = act ? (sinb ? x0 * cs + xp * sn : x0 * cs - xp * sn) : 0.0;
        const double y0 = wsum(am * v0 * w), y1 = wsum(am * v1 * w);
        const double g0 = M.gi[0][0] * y0 + M.gi[0][1] * y1, g1 = M.gi[1][0] * y0 + M.gi[1][1] * y1;
        const double e = w - (v0 * g0 + v1 * g1);
        const double h = am * e;
        const double qf = wsum(h * e) + g0 * g0 + g1 * g1;
        const double hp = __shfl(h, partner, 64);
        // d qf_j / d x = 2 R_j (A e): the shift of A e back by +phi_j
        const double dqj = 2.0 * (sinb ? cs * h - sn * hp : cs * h + sn * hp);
        const double l = -0.5 * M.logdetL0 - K * log(qf);
        const double gl = act ? (-K / qf) * dqj : 0.0;
        if (uniform(l > mx)) {
            const double r = exp(mx - l);
            se = se * r + 1.0;
            G = G * r + gl;
            mx = l;
        } else {
            const double r = exp(l - mx);
            se += r;
            G += r * gl;
        }
    }
    const double lnet = mx + log(se) - log(32.0);
    const double lg = M.lng - K * log1p(M.gc * t);
    const double A = M.log_eps + lg, B = M.log_1m_eps + lnet;
    const double hi = A > B ? A : B;
    const double lm = hi + log(exp(A - hi) + exp(B - hi));
    const double wg = exp(A - lm), wn = exp(B - lm);
    dq = act ? wg * (-K * M.gc / (1.0 + M.gc * t)) * 2.0 * k * k * x0 + wn * (G / se) : 0.0;
    return lm;
}

// phi at the unit vector x (lane l holds coordinates l + 64 c, c < C) and its
// tangent gradient g.  Sums over a lane's coordinates run in the order c = 0,
// 1, ..., so C = 4 gives K <= 64 the bits of C = 2 (the extra terms are zeros).
template <int C>
__device__ double plan_eval(const PlanPoint &P, const PlanMix *mix, double *xs, double *us, const double *ct,
                            int lane, const double (&x)[C], double (&g)[C])
{
    const int K = P.K, N = P.N, n2 = 2 * K, q = N / 4;
    bool v[C];
    int kk[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int m = lane + 64 * c;
        v[c] = m < n2;
        kk[c] = m % K + 1;
        if (v[c]) xs[m] = x[c];
    }
    wave_sync_lds();
    double tl = v[0] ? (double)kk[0] * kk[0] * x[0] * x[0] : 0.0;
#pragma unroll
    for (int c = 1; c < C; ++c) tl += v[c] ? (double)kk[c] * kk[c] * x[c] * x[c] : 0.0;
    const double t = wsum(tl);
    double s3 = 0.0;
#pragma unroll
    for (int r = 0; r < 2 * C; ++r) {  // grid points lane + 64 r (N <= 128 C)
        const int j = lane + 64 * r;
        if (j < N) {
            double u = 0.0;
            int ic = 0;
            for (int k = 1; k <= K; ++k) {
                ic += j;
                if (ic >= N) ic -= N;
                int is = ic - q;
                if (is < 0) is += N;
                const double term = xs[k - 1] * ct[ic] + xs[K + k - 1] * ct[is];
                u += (k & 1) ? -term : term;
            }
            us[j] = u * u;
            s3 += u * u * u;
        }
    }
    const double S3 = wsum(s3);
    wave_sync_lds();
    auto dh = [&](int m) {
        const int k = m % K + 1;
        const int off = m >= K ? q : 0;
        double acc = 0.0;
        int ic = 0;
        for (int j = 0; j < N; ++j) {
            int idx = ic - off;
            if (idx < 0) idx += N;
            acc += us[j] * ct[idx];
            ic += k;
            if (ic >= N) ic -= N;
        }
        return (k & 1) ? -acc : acc;
    };
    double val = P.dt0 * t + P.cH * (kPiP / (3.0 * N)) * P.amp3 * S3;
    double dt = P.dt0;
    if (P.sigma) {
        val += K * log1p(P.a * t);
        dt += K * P.a / (1.0 + P.a * t);
    }
    const double cg = P.cH * kPiP * P.amp3 / N;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const double d = v[c] ? dh(lane + 64 * c) : 0.0;
        g[c] = v[c] ? dt * 2.0 * kk[c] * kk[c] * x[c] + cg * d : 0.0;
    }
    if constexpr (C == 2) {
        if (mix) {  // phi = log f - log q_mix (K <= 32: coordinate `lane` only)
            double dq;
            val -= mix_log_q(*mix, K, lane, x[0], t, dq);
            g[0] -= dq;
        }
    }
    double gxl = g[0] * x[0];
#pragma unroll
    for (int c = 1; c < C; ++c) gxl += g[c] * x[c];
    const double gx = wsum(gxl);
#pragma unroll
    for (int c = 0; c < C; ++c) g[c] -= gx * x[c];
    wave_sync_lds();  // the next evaluation overwrites xs and us
    return val;
}

// Lane sums of a . b over the lane's C coordinates, in the order c = 0, 1, ...
template <int C>
__device__ __forceinline__ double dotl(const double (&a)[C], const double (&b)[C])
{
    double s = a[0] * b[0];
#pragma unroll
    for (int c = 1; c < C; ++c) s += a[c] * b[c];
    return s;
}

template <int C>
__global__ void __launch_bounds__(64 * kPlanWaves) k_plan_search(PlanArgs a)
{
    __shared__ double xs_all[kPlanWaves][64 * C];
    __shared__ double us_all[kPlanWaves][128 * C];
    __shared__ double ct_all[kPlanWaves][128 * C];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int item = blockIdx.x * kPlanWaves + w;
    if (item >= a.n_items) return;  // whole wave; no workgroup barrier follows
    const int per = a.n_starts + a.n_user;
    const int p = item / per, s = item % per;
    const PlanPoint P = a.pts[p];
    const PlanMix *M = a.mix ? a.mix + p : nullptr;
    double *xs = xs_all[w], *us = us_all[w], *ct = ct_all[w];
    const int K = P.K, N = P.N, n2 = 2 * K;
    for (int r = lane; r < N; r += 64) ct[r] = cos(2.0 * kPiP * r / N);
    double x[C];
    if (s >= a.n_starts) {  // a caller start
        const double *u = a.x_user + ((size_t)p * a.n_user + (s - a.n_starts)) * kPlanStride;
#pragma unroll
        for (int c = 0; c < C; ++c) x[c] = lane + 64 * c < n2 ? u[lane + 64 * c] : 0.0;
    } else if (s == 0) {  // zero-mean Dirichlet kernel: equal cos coefficients
#pragma unroll
        for (int c = 0; c < C; ++c) x[c] = lane + 64 * c < K ? 1.0 : 0.0;
    } else if (s == 1) {  // all energy in mode 1
#pragma unroll
        for (int c = 0; c < C; ++c) x[c] = lane + 64 * c == 0 ? 1.0 : 0.0;
    } else {  // independent normal coordinates, Box-Muller pairs of Philox words
        auto normal = [&](int m) {
            const uint4 wd = philox4x32_10((uint32_t)s, P.point_id, (uint32_t)(m >> 1), 0x504C414Eu, a.seed_lo,
                                           a.seed_hi);
            const double u1 = ((double)wd.x + 0.5) * 0x1p-32, u2 = ((double)wd.y + 0.5) * 0x1p-32;
            const double r = sqrt(-2.0 * log(u1)), th = 2.0 * kPiP * u2;
            return (m & 1) ? r * sin(th) : r * cos(th);
        };
#pragma unroll
        for (int c = 0; c < C; ++c) x[c] = lane + 64 * c < n2 ? normal(lane + 64 * c) : 0.0;
    }
    {
        const double r = sqrt(wsum(dotl<C>(x, x)));
#pragma unroll
        for (int c = 0; c < C; ++c) x[c] /= r;
    }
    wave_sync_lds();  // cos table
    double g[C];
    double f = plan_eval<C>(P, M, xs, us, ct, lane, x, g);
    int evals = 1;
    // curvature pairs, newest first: s = x_new - x_old, y = g_old - g_new
    double S[kPlanMem][C], Y[kPlanMem][C], RHO[kPlanMem];
#pragma unroll
    for (int i = 0; i < kPlanMem; ++i) {
        RHO[i] = 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) S[i][c] = Y[i][c] = 0.0;
    }
    int mc = 0;
    double gamma = 1.0;
    for (int it = 0; it < kPlanMaxIter; ++it) {
        const double gn = sqrt(wsum(dotl<C>(g, g)));
        if (uniform(!(gn > 1e-13 * (1.0 + fabs(f))))) break;
        // two-loop recursion on the ascent problem: d = H g
        double qv[C], al[kPlanMem];
#pragma unroll
        for (int c = 0; c < C; ++c) qv[c] = g[c];
#pragma unroll
        for (int i = 0; i < kPlanMem; ++i) {
            al[i] = 0.0;
            if (i < mc) {
                al[i] = RHO[i] * wsum(dotl<C>(S[i], qv));
#pragma unroll
                for (int c = 0; c < C; ++c) qv[c] -= al[i] * Y[i][c];
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) qv[c] *= gamma;
#pragma unroll
        for (int i = kPlanMem - 1; i >= 0; --i) {
            if (i < mc) {
                const double b = RHO[i] * wsum(dotl<C>(Y[i], qv));
#pragma unroll
                for (int c = 0; c < C; ++c) qv[c] += S[i][c] * (al[i] - b);
            }
        }
        double d[C];
#pragma unroll
        for (int c = 0; c < C; ++c) d[c] = qv[c];
        double slope = wsum(dotl<C>(d, g));
        double step = 1.0;
        if (uniform(!(slope > 0.0)) || mc == 0) {  // steepest ascent, at most half a radian
#pragma unroll
            for (int c = 0; c < C; ++c) d[c] = g[c];
            slope = gn * gn;
            mc = 0;
            gamma = 1.0;
            step = fmin(1.0, 0.5 / gn);
        }
        double f2 = f, x2[C], g2[C];
        bool ok = false;
        for (int ls = 0; ls < kPlanMaxBacktrack; ++ls) {
#pragma unroll
            for (int c = 0; c < C; ++c) x2[c] = x[c] + step * d[c];
            const double r = sqrt(wsum(dotl<C>(x2, x2)));
#pragma unroll
            for (int c = 0; c < C; ++c) x2[c] /= r;
            f2 = plan_eval<C>(P, M, xs, us, ct, lane, x2, g2);
            ++evals;
            if (uniform(f2 >= f + 1e-4 * step * slope)) {
                ok = true;
                break;
            }
            step *= 0.5;
        }
        if (!ok) break;
        double sx[C], yv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            sx[c] = x2[c] - x[c];
            yv[c] = g[c] - g2[c];
        }
        const double sy = wsum(dotl<C>(sx, yv)), yy = wsum(dotl<C>(yv, yv));
        const double gain = f2 - f;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            x[c] = x2[c];
            g[c] = g2[c];
        }
        f = f2;
        if (uniform(sy > 1e-300 && yy > 0.0)) {
#pragma unroll
            for (int i = kPlanMem - 1; i > 0; --i) {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    S[i][c] = S[i - 1][c];
                    Y[i][c] = Y[i - 1][c];
                }
                RHO[i] = RHO[i - 1];
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                S[0][c] = sx[c];
                Y[0][c] = yv[c];
            }
            RHO[0] = 1.0 / sy;
            gamma = sy / yy;
            mc = mc < kPlanMem ? mc + 1 : kPlanMem;
        }
        if (uniform(gain < 1e-16 * (1.0 + fabs(f)) && it > 5)) break;
    }
    double *xo = a.xbest + (size_t)item * kPlanStride;
#pragma unroll
    for (int c = 0; c < C; ++c) xo[lane + 64 * c] = lane + 64 * c < n2 ? x[c] : 0.0;
    if (lane == 0) {
        a.val[item] = f;
        a.evals[item] = evals;
    }
}

}  // namespace

hipError_t launch_plan_search(const PlanArgs &a, int max_K, hipStream_t st)
{
    if (a.n_items <= 0) return hipSuccess;
    if (max_K > kPlanStride / 2) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)((a.n_items + kPlanWaves - 1) / kPlanWaves);
    if (max_K <= 64) hipLaunchKernelGGL(k_plan_search<2>, dim3(grid), dim3(64 * kPlanWaves), 0, st, a);
    else hipLaunchKernelGGL(k_plan_search<4>, dim3(grid), dim3(64 * kPlanWaves), 0, st, a);
    return hipGetLastError();
}

}  // namespace tkdv
