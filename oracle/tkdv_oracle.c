/*
 * tkdv_oracle.c -- plain CPU FP64 oracle for rejection sampling of the
 * truncated-KdV (TKdV) Gibbs measure on the energy sphere S^{2K-1}
 * (N. J. Moore & B. Foerster, "In search of rogue waves: a novel proposal
 * distribution for parallelized rejection sampling of the truncated KdV Gibbs
 * measure", arXiv 2411.16952).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the HIP library; both sides
 * implement the same counter-based generator (Philox4x32-10) from its
 * published definition, so that individual proposals can be compared.
 *
 * Everything is computed in IEEE double precision, one proposal at a time, in
 * the order the paper's algorithm (Sec. IV.B, steps 2-4) states it:
 *   draw X ~ gamma_Sigma (or the standard Gaussian for the uniform proposal),
 *   project X^ = X/|X|, evaluate H2 by Parseval and H3 by the O(K^2) double
 *   sum, form f/(M g) and accept with that probability.
 * There is no blocking, fusion or reordering of the per-proposal arithmetic.
 * Proposals are independent (Sec. IV.B, closing paragraph); the only
 * parallelism here is an OpenMP loop over proposal indices whose results are
 * written to per-index slots, so the output does not depend on the thread
 * count.  Statistics are accumulated afterwards in increasing proposal index.
 *
 * Conventions fixed by this implementation (the paper is silent on them):
 *   - coordinate layout x^ = [x^_1..x^_K | x^_{K+1}..x^_{2K}] (cos | sin
 *     block), so that u^_k = sqrt(E0/2pi)(x^_k - i x^_{K+k}) (Sec. II.C);
 *   - random numbers: Philox4x32-10, key = (seed_lo, seed_hi), counter =
 *     (i_lo, i_hi, point_id, block | tag<<16); proposal i consumes words
 *     0..2K+1 of blocks 0..ceil((2K+2)/4)-1; word w -> U = (w + 1/2) 2^-32;
 *     words (2m, 2m+1) -> Box-Muller pair (z_2m, z_2m+1); word 2K is the
 *     acceptance uniform, word 2K+1 is reserved for a mixture component draw;
 *   - accept iff log U < log a (strict).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Threads of one parallel loop: nthreads if positive, else the OpenMP
   default.  The choice applies to that loop only, so a one-thread call leaves
   no process-wide setting behind. */
static inline int orc_threads(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

#define ORC_KMAX 128
#define ORC_NBINS 64

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11).  Two 32x32->64 multiplications per round with  */
/* the multipliers below, the key bumped by the two Weyl constants between  */
/* rounds, ten rounds.                                                      */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_MUL_A = 0xD2511F53u;
static const uint32_t PHILOX_MUL_B = 0xCD9E8D57u;
static const uint32_t PHILOX_WEYL_A = 0x9E3779B9u;
static const uint32_t PHILOX_WEYL_B = 0xBB67AE85u;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod_a = (uint64_t)PHILOX_MUL_A * (uint64_t)x0;
        uint64_t prod_b = (uint64_t)PHILOX_MUL_B * (uint64_t)x2;
        uint32_t hi_a = (uint32_t)(prod_a >> 32), lo_a = (uint32_t)prod_a;
        uint32_t hi_b = (uint32_t)(prod_b >> 32), lo_b = (uint32_t)prod_b;
        uint32_t y0 = hi_b ^ x1 ^ k0;
        uint32_t y1 = lo_b;
        uint32_t y2 = hi_a ^ x3 ^ k1;
        uint32_t y3 = lo_a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHILOX_WEYL_A;
        k1 += PHILOX_WEYL_B;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Words 0..nwords-1 of proposal i of point point_id under the given tag. */
void orc_proposal_words(uint64_t seed, uint64_t i, uint32_t point_id, uint32_t tag,
                        int nwords, uint32_t *words)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int nblocks = (nwords + 3) / 4;
    for (int b = 0; b < nblocks; ++b) {
        uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), point_id,
                           (uint32_t)b | (tag << 16)};
        uint32_t out[4];
        orc_philox4x32_10(ctr, key, out);
        for (int w = 0; w < 4 && 4 * b + w < nwords; ++w) words[4 * b + w] = out[w];
    }
}

/* Open-interval uniform from one 32-bit word: (w + 1/2) 2^-32, never 0 or 1. */
double orc_uniform(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

/*
 * The 2K standard normals z and the two extra uniforms of proposal i.
 * Box-Muller on word pairs: r = sqrt(-2 ln U1), z_2m = r cos(2 pi U2),
 * z_2m+1 = r sin(2 pi U2).  u_accept = U(word 2K), u_mix = U(word 2K+1).
 */
void orc_normals(uint64_t seed, uint64_t i, uint32_t point_id, int K, double *z,
                 double *u_accept, double *u_mix)
{
    uint32_t words[2 * ORC_KMAX + 4];
    int nw = 2 * K + 2;
    orc_proposal_words(seed, i, point_id, 0u, nw, words);
    for (int m = 0; m < K; ++m) {
        double u1 = orc_uniform(words[2 * m]);
        double u2 = orc_uniform(words[2 * m + 1]);
        double r = sqrt(-2.0 * log(u1));
        double th = 2.0 * M_PI * u2;
        z[2 * m] = r * cos(th);
        z[2 * m + 1] = r * sin(th);
    }
    if (u_accept) *u_accept = orc_uniform(words[2 * K]);
    if (u_mix) *u_mix = orc_uniform(words[2 * K + 1]);
}

/* ------------------------------------------------------------------------ */
/* Proposal parameters (Sec. III.A): sigma_k^2 = 1/(1 + alpha beta' k^2/K^3) */
/* for the anisotropic Gaussian gamma_Sigma, Sigma = diag(s^2, s^2).         */
/* ------------------------------------------------------------------------ */
double orc_sigma2(int K, double beta_p, double alpha, int k)
{
    double K3 = (double)K * K * K;
    return 1.0 / (1.0 + alpha * beta_p * (double)k * k / K3);
}

/* F(alpha) = 1 - (alpha/K) sum_k 1/(1 + alpha beta' k^2/K^3)  (Sec. III.A). */
double orc_F_alpha(int K, double beta_p, double alpha)
{
    double s = 0.0;
    for (int k = 1; k <= K; ++k) s += orc_sigma2(K, beta_p, alpha, k);
    return 1.0 - alpha / K * s;
}

/* ------------------------------------------------------------------------ */
/* Hamiltonian pieces on the sphere.                                        */
/* ------------------------------------------------------------------------ */

/* t = sum_k k^2 (x^_k^2 + x^_{K+k}^2); H2 = E0 t  (Sec. III.A, Parseval). */
double orc_t(int K, const double *xh)
{
    double t = 0.0;
    for (int k = 1; k <= K; ++k) {
        double s = xh[k - 1] * xh[k - 1] + xh[K + k - 1] * xh[K + k - 1];
        t += (double)k * k * s;
    }
    return t;
}

double orc_H2(int K, double E0, const double *xh) { return E0 * orc_t(K, xh); }

/*
 * H3 by the double sum of Sec. IV.A:
 *   H3 = 2 pi sum_{n=1..K} Re( conj(u^_n) sum_{k=1..n-1} u^_k u^_{n-k} ),
 * with u^_k = sqrt(E0/2pi)(x^_k - i x^_{K+k}) (Sec. II.C).
 */
double orc_H3_triad(int K, double E0, const double *xh)
{
    double a = sqrt(E0 / (2.0 * M_PI));
    double total = 0.0;
    for (int n = 1; n <= K; ++n) {
        double in_re = 0.0, in_im = 0.0;
        for (int k = 1; k <= n - 1; ++k) {
            double p_re = a * xh[k - 1], p_im = -a * xh[K + k - 1];
            double q_re = a * xh[n - k - 1], q_im = -a * xh[K + n - k - 1];
            in_re += p_re * q_re - p_im * q_im;
            in_im += p_re * q_im + p_im * q_re;
        }
        double n_re = a * xh[n - 1], n_im = -a * xh[K + n - 1];
        /* Re(conj(u_n) * inner) */
        total += n_re * in_re + n_im * in_im;
    }
    return 2.0 * M_PI * total;
}

/*
 * Surface displacement on the grid xi_j = -pi + 2 pi j/N, j = 0..N-1:
 *   u(xi) = sum_k a_k cos(k xi) + b_k sin(k xi), a_k = 2 Re u^_k, b_k = -2 Im u^_k
 * (Sec. II.B), i.e. u = sqrt(2 E0/pi) sum_k (x^_k cos k xi + x^_{K+k} sin k xi).
 */
void orc_grid(int K, double E0, int N, const double *xh, double *u)
{
    double amp = sqrt(2.0 * E0 / M_PI);
    for (int j = 0; j < N; ++j) {
        double xi = -M_PI + 2.0 * M_PI * (double)j / (double)N;
        double s = 0.0;
        for (int k = 1; k <= K; ++k)
            s += xh[k - 1] * cos(k * xi) + xh[K + k - 1] * sin(k * xi);
        u[j] = amp * s;
    }
}

/*
 * H3 = (1/6) int u^3 dxi by the N-point trapezoid rule on the periodic grid
 * (definition of H3, Sec. II.A).  Exact when N >= 3K+1 because u^3 is a
 * trigonometric polynomial of degree 3K.
 */
double orc_H3_quad(int K, double E0, int N, const double *xh)
{
    double *u = (double *)malloc(sizeof(double) * (size_t)N);
    orc_grid(K, E0, N, xh, u);
    double s = 0.0;
    for (int j = 0; j < N; ++j) s += u[j] * u[j] * u[j];
    free(u);
    return (1.0 / 6.0) * (2.0 * M_PI / N) * s;
}

/* beta H_K = beta'/(E0 K^2) (H2 - (C3/C2) H3)   (Sec. IV.A). */
double orc_beta_H(int K, double E0, double beta_p, double c32, const double *xh)
{
    double H2 = orc_H2(K, E0, xh);
    double H3 = orc_H3_triad(K, E0, xh);
    return beta_p / (E0 * (double)K * K) * (H2 - c32 * H3);
}

/*
 * log of the unnormalised ratio target/proposal on the sphere.
 *   proposal 0 (uniform mu0):  log f = -beta H_K
 *   proposal 1 (Sigma):        log f/g = -beta H_K + K log(1 + alpha* beta' t/K^3)
 * (Sec. IV.A, ratio f/g with Const = 1/Z).
 */
double orc_log_ratio(int K, double E0, double beta_p, double c32, double alpha,
                     int proposal, const double *xh)
{
    double lr = -orc_beta_H(K, E0, beta_p, c32, xh);
    if (proposal == 1) {
        double K3 = (double)K * K * K;
        lr += K * log1p(alpha * beta_p * orc_t(K, xh) / K3);
    }
    return lr;
}

/* Same, for an arbitrary non-zero y in R^{2K} projected to the sphere. */
double orc_log_ratio_unnorm(int K, double E0, double beta_p, double c32, double alpha,
                            int proposal, const double *y)
{
    double xh[2 * ORC_KMAX];
    double r2 = 0.0;
    for (int m = 0; m < 2 * K; ++m) r2 += y[m] * y[m];
    double r = sqrt(r2);
    for (int m = 0; m < 2 * K; ++m) xh[m] = y[m] / r;
    return orc_log_ratio(K, E0, beta_p, c32, alpha, proposal, xh);
}

/* ------------------------------------------------------------------------ */
/* One proposal: draw, project, evaluate (Sec. IV.B steps 2-4).             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t K;
    int32_t N;          /* grid points for the statistics                   */
    int32_t proposal;   /* 0 uniform, 1 Sigma                                */
    uint32_t point_id;  /* third counter word                                */
    double E0, beta_p, c32;
    double alpha_star;  /* root of F (Sigma proposal only)                   */
    double log_M;       /* log of the rejection constant                     */
    uint64_t seed;
} orc_point;

/* x^ of proposal i; returns log a = log f/(M g) and the acceptance log U. */
double orc_proposal(const orc_point *p, uint64_t i, double *xh, double *log_u)
{
    int K = p->K;
    double z[2 * ORC_KMAX];
    double x[2 * ORC_KMAX];
    double u_acc;
    orc_normals(p->seed, i, p->point_id, K, z, &u_acc, NULL);
    for (int m = 0; m < 2 * K; ++m) {
        double scale = 1.0;
        if (p->proposal == 1) scale = sqrt(orc_sigma2(K, p->beta_p, p->alpha_star, m % K + 1));
        x[m] = scale * z[m];
    }
    double r2 = 0.0;
    for (int m = 0; m < 2 * K; ++m) r2 += x[m] * x[m];
    double r = sqrt(r2);
    for (int m = 0; m < 2 * K; ++m) xh[m] = x[m] / r;
    if (log_u) *log_u = log(u_acc);
    return orc_log_ratio(K, p->E0, p->beta_p, p->c32, p->alpha_star, p->proposal, xh) - p->log_M;
}

/* ------------------------------------------------------------------------ */
/* Learned proposal (not in the paper): a defensive mixture                 */
/*   q_mix = eps g_Sigma + (1 - eps) q_net,  q_net = (1/S) sum_j ACG_j,      */
/* of angular central Gaussian densities w.r.t. mu0, exactly normalised:     */
/*   ACG(x^; L) = |L|^{-1/2} (x^T L^{-1} x^)^{-K}   (x^ in S^{2K-1}).        */
/* g_Sigma is the paper's proposal, an ACG with L = Sigma (Sec. III.B).      */
/* Component j is the base L0 = D + V V^T (D = diag(d_k) on the cos and sin */
/* coordinate of mode k, V of rank R) rotated by the xi-shift phi_j =       */
/* 2 pi j/S, which rotates mode k by the angle k phi_j; f is invariant      */
/* under these shifts.                                                      */
/* ------------------------------------------------------------------------ */
#define ORC_MIX_S 32
#define ORC_MIX_R 2

typedef struct {
    int32_t K;
    int32_t pad;
    double eps;                          /* weight of g_Sigma                   */
    double logd[ORC_KMAX];               /* log d_k, k = 1..K                   */
    double V[2 * ORC_KMAX][ORC_MIX_R];   /* rows = coordinates                  */
} orc_mixture;

/* Integer threshold of the g_Sigma component, E = S floor(eps 2^32 / S), and
   the weight it realises, eps_eff = E 2^-32 (used in every density). */
uint64_t orc_mix_threshold(const orc_mixture *m)
{
    return (uint64_t)ORC_MIX_S * (uint64_t)floor(m->eps * (double)(1ull << 32) / ORC_MIX_S);
}
double orc_mix_eps(const orc_mixture *m) { return ldexp((double)orc_mix_threshold(m), -32); }

/* (R_phi x)_k = x_k cos k phi + x_{K+k} sin k phi,
   (R_phi x)_{K+k} = x_{K+k} cos k phi - x_k sin k phi  (shift of u by phi). */
void orc_shift(int K, double phi, const double *x, double *out)
{
    for (int k = 1; k <= K; ++k) {
        double c = cos(k * phi), s = sin(k * phi);
        double a = x[k - 1], b = x[K + k - 1];
        out[k - 1] = a * c + b * s;
        out[K + k - 1] = b * c - a * s;
    }
}

/* r x r Gram G = I + V^T D^-1 V, its inverse and log det (r = 2, closed form). */
static void mix_gram(const orc_mixture *m, double Ginv[ORC_MIX_R][ORC_MIX_R], double *logdetG)
{
    int K = m->K;
    double G[ORC_MIX_R][ORC_MIX_R] = {{1.0, 0.0}, {0.0, 1.0}};
    for (int c = 0; c < 2 * K; ++c) {
        double a = exp(-m->logd[c % K]);
        for (int p = 0; p < ORC_MIX_R; ++p)
            for (int q = 0; q < ORC_MIX_R; ++q) G[p][q] += m->V[c][p] * a * m->V[c][q];
    }
    double det = G[0][0] * G[1][1] - G[0][1] * G[1][0];
    Ginv[0][0] = G[1][1] / det;
    Ginv[1][1] = G[0][0] / det;
    Ginv[0][1] = -G[0][1] / det;
    Ginv[1][0] = -G[1][0] / det;
    *logdetG = log(det);
}

/* log ACG(w; L0) for a point w of the sphere, via x^T L0^-1 x = e^T D^-1 e + |g|^2,
   g = G^-1 V^T D^-1 w, e = w - V g (Woodbury, no cancellation). */
static double mix_log_acg0(const orc_mixture *m, const double Ginv[ORC_MIX_R][ORC_MIX_R],
                           double logdet_L0, const double *w)
{
    int K = m->K;
    double y[ORC_MIX_R] = {0.0, 0.0};
    for (int c = 0; c < 2 * K; ++c) {
        double a = exp(-m->logd[c % K]);
        for (int p = 0; p < ORC_MIX_R; ++p) y[p] += m->V[c][p] * a * w[c];
    }
    double g[ORC_MIX_R];
    for (int p = 0; p < ORC_MIX_R; ++p) g[p] = Ginv[p][0] * y[0] + Ginv[p][1] * y[1];
    double qf = g[0] * g[0] + g[1] * g[1];
    for (int c = 0; c < 2 * K; ++c) {
        double e = w[c] - (m->V[c][0] * g[0] + m->V[c][1] * g[1]);
        qf += exp(-m->logd[c % K]) * e * e;
    }
    return -0.5 * logdet_L0 - K * log(qf);
}

/* log q_net and log q_mix at x^ (normalised densities w.r.t. mu0).
   log g_Sigma = sum_k log(1 + alpha beta' k^2/K^3) - K log(1 + alpha beta' t/K^3). */
void orc_mix_log_q(const orc_point *p, const orc_mixture *m, const double *xh,
                   double *log_q_net, double *log_q_mix)
{
    int K = p->K;
    double Ginv[ORC_MIX_R][ORC_MIX_R], ldG;
    mix_gram(m, Ginv, &ldG);
    double ldD = 0.0;
    for (int k = 0; k < K; ++k) ldD += 2.0 * m->logd[k];
    double logdet_L0 = ldD + ldG;
    double terms[ORC_MIX_S], mx = -INFINITY;
    double w[2 * ORC_KMAX];
    for (int j = 0; j < ORC_MIX_S; ++j) {
        /* ACG_j(x^) = ACG(R_j^T x^; L0), R_j^T = shift by -phi_j */
        orc_shift(K, -2.0 * M_PI * j / ORC_MIX_S, xh, w);
        terms[j] = mix_log_acg0(m, Ginv, logdet_L0, w);
        if (terms[j] > mx) mx = terms[j];
    }
    double se = 0.0;
    for (int j = 0; j < ORC_MIX_S; ++j) se += exp(terms[j] - mx);
    double lnet = mx + log(se) - log((double)ORC_MIX_S);
    double K3 = (double)K * K * K, lng = 0.0;
    for (int k = 1; k <= K; ++k) lng += log1p(p->alpha_star * p->beta_p * (double)k * k / K3);
    double lg = lng - K * log1p(p->alpha_star * p->beta_p * orc_t(K, xh) / K3);
    double eps = orc_mix_eps(m);
    double a = log(eps) + lg, b = log1p(-eps) + lnet;
    double hi = a > b ? a : b;
    if (log_q_net) *log_q_net = lnet;
    if (log_q_mix) *log_q_mix = hi + log(exp(a - hi) + exp(b - hi));
}

/*
 * Draw of proposal i from q_mix.  Words 0..2K-1: the 2K normals zeta (as for
 * the paper's proposal); word 2K: acceptance uniform; word 2K+1: component
 * word w_c; words (2K+2, 2K+3): one Box-Muller pair eta (r = 2).
 * The component is chosen in integers: w_c < E gives g_Sigma with
 * X = Sigma^{1/2} zeta, otherwise j = (w_c - E) div B with B = (2^32 - E)/S
 * and X = D^{1/2} zeta + (R_j V) eta ~ N(0, R_j L0 R_j^T).  x^ = X/|X|.
 * E = S floor(eps 2^32/S), so the mixture weights are exactly E 2^-32 and
 * (1 - E 2^-32)/S (orc_mix_eps).  Returns the component (-1 for g_Sigma)
 * and log U.
 */
int orc_mix_draw(const orc_point *p, const orc_mixture *m, uint64_t i, double *xh, double *log_u)
{
    int K = p->K;
    uint32_t words[2 * ORC_KMAX + 4];
    orc_proposal_words(p->seed, i, p->point_id, 0u, 2 * K + 4, words);
    double z[2 * ORC_KMAX];
    for (int q = 0; q < K; ++q) {
        double u1 = orc_uniform(words[2 * q]), u2 = orc_uniform(words[2 * q + 1]);
        double r = sqrt(-2.0 * log(u1)), th = 2.0 * M_PI * u2;
        z[2 * q] = r * cos(th);
        z[2 * q + 1] = r * sin(th);
    }
    uint64_t wc = words[2 * K + 1], E = orc_mix_threshold(m), B = ((1ull << 32) - E) / ORC_MIX_S;
    double e1 = orc_uniform(words[2 * K + 2]), e2 = orc_uniform(words[2 * K + 3]);
    double er = sqrt(-2.0 * log(e1)), eth = 2.0 * M_PI * e2;
    double eta[2] = {er * cos(eth), er * sin(eth)};
    if (log_u) *log_u = log(orc_uniform(words[2 * K]));
    double X[2 * ORC_KMAX];
    int comp = -1;
    if (wc < E) {
        for (int c = 0; c < 2 * K; ++c) X[c] = sqrt(orc_sigma2(K, p->beta_p, p->alpha_star, c % K + 1)) * z[c];
    } else {
        comp = (int)((wc - E) / B);
        double v0[2 * ORC_KMAX], v1[2 * ORC_KMAX], rv0[2 * ORC_KMAX], rv1[2 * ORC_KMAX];
        for (int c = 0; c < 2 * K; ++c) { v0[c] = m->V[c][0]; v1[c] = m->V[c][1]; }
        double phi = 2.0 * M_PI * comp / ORC_MIX_S;
        orc_shift(K, phi, v0, rv0);
        orc_shift(K, phi, v1, rv1);
        for (int c = 0; c < 2 * K; ++c)
            X[c] = exp(0.5 * m->logd[c % K]) * z[c] + rv0[c] * eta[0] + rv1[c] * eta[1];
    }
    double r2 = 0.0;
    for (int c = 0; c < 2 * K; ++c) r2 += X[c] * X[c];
    double r = sqrt(r2);
    for (int c = 0; c < 2 * K; ++c) xh[c] = X[c] / r;
    return comp;
}

/* log a = log f - log q_mix - log M_mix for proposal i of the mixture sampler
   (p->log_M holds log M_mix for the normalised q_mix). */
double orc_mix_proposal(const orc_point *p, const orc_mixture *m, uint64_t i, double *xh, double *log_u)
{
    orc_mix_draw(p, m, i, xh, log_u);
    double lqm;
    orc_mix_log_q(p, m, xh, NULL, &lqm);
    return -orc_beta_H(p->K, p->E0, p->beta_p, p->c32, xh) - lqm - p->log_M;
}

/* The rejection sampler with the mixture proposal over [i0, i0+n): accept
   flags, optional log a / log U, accepted rows (up to cap) and statistics. */
uint64_t orc_mix_sample(const orc_point *p, const orc_mixture *m, uint64_t i0, uint64_t n,
                        uint8_t *accept, double *log_a_out, double *log_u_out, double *xhat_out,
                        uint64_t *index_out, uint64_t cap, int nthreads);

/* ------------------------------------------------------------------------ */
/* Statistics of the accepted ensemble (moments of u pooled over samples x  */
/* grid points, exceedance of 2 sigma with sigma = sqrt(E0/pi), histogram of */
/* u(0) on [-u_max, u_max], u_max = sqrt(2 K E0/pi)), and the extremes of    */
/* Sec. V.D: grid values above 4 sigma, samples whose largest grid value is  */
/* above 4 sigma, and the largest displacement with its sample's index      */
/* (the lowest index among equal maxima).                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t n_proposed, n_accepted, n_written, n_violations, n_exceed, n_grid;
    double max_log_a;
    double S1, S2, S3, S4;
    double skewness, kurtosis, p_exceed;
    double hist_lo, hist_hi;
    uint64_t hist[ORC_NBINS];
    uint64_t n_exceed4, n_max4; /* grid values > 4 sigma; samples with max_j u_j > 4 sigma */
    double peak_u;              /* largest u over samples x grid (-inf: no sample)        */
    uint64_t peak_index;        /* index of the sample attaining it (UINT64_MAX: none)    */
} orc_stats;

typedef struct {
    int K, N;
    double E0, amp, two_sigma, four_sigma, u_max;
    double *cosv, *sinv; /* [N][K] */
} orc_grid_table;

static void grid_table_init(orc_grid_table *g, int K, int N, double E0)
{
    g->K = K; g->N = N; g->E0 = E0;
    g->amp = sqrt(2.0 * E0 / M_PI);
    g->two_sigma = 2.0 * sqrt(E0 / M_PI);
    g->four_sigma = 4.0 * sqrt(E0 / M_PI);
    g->u_max = sqrt(2.0 * K * E0 / M_PI);
    g->cosv = (double *)malloc(sizeof(double) * (size_t)N * K);
    g->sinv = (double *)malloc(sizeof(double) * (size_t)N * K);
    for (int j = 0; j < N; ++j) {
        double xi = -M_PI + 2.0 * M_PI * (double)j / (double)N;
        for (int k = 1; k <= K; ++k) {
            g->cosv[(size_t)j * K + k - 1] = cos(k * xi);
            g->sinv[(size_t)j * K + k - 1] = sin(k * xi);
        }
    }
}

static void grid_table_free(orc_grid_table *g) { free(g->cosv); free(g->sinv); }

int orc_hist_bin(double u0, double u_max)
{
    double pos = (u0 + u_max) / (2.0 * u_max) * ORC_NBINS;
    int b = (int)floor(pos);
    if (b < 0) b = 0;
    if (b > ORC_NBINS - 1) b = ORC_NBINS - 1;
    return b;
}

static void stats_init(orc_stats *st, const orc_grid_table *g)
{
    memset(st, 0, sizeof(*st));
    st->hist_lo = -g->u_max;
    st->hist_hi = g->u_max;
    st->peak_u = -INFINITY;
    st->peak_index = UINT64_MAX;
}

/* One accepted sample x^ (proposal index `index`); samples come in increasing
   index, so a later sample replaces the peak only with a strictly larger u. */
static void stats_add_sample(orc_stats *st, const orc_grid_table *g, const double *xh, uint64_t index)
{
    int K = g->K;
    double umax = -INFINITY;
    for (int j = 0; j < g->N; ++j) {
        double s = 0.0;
        for (int k = 0; k < K; ++k)
            s += xh[k] * g->cosv[(size_t)j * K + k] + xh[K + k] * g->sinv[(size_t)j * K + k];
        double u = g->amp * s;
        double u2 = u * u;
        st->S1 += u;
        st->S2 += u2;
        st->S3 += u2 * u;
        st->S4 += u2 * u2;
        if (u > g->two_sigma) st->n_exceed++;
        if (u > g->four_sigma) st->n_exceed4++;
        if (u > umax) umax = u;
    }
    if (umax > g->four_sigma) st->n_max4++;
    if (umax > st->peak_u) {
        st->peak_u = umax;
        st->peak_index = index;
    }
    st->n_grid += (uint64_t)g->N;
    /* u(0): xi = 0 is a grid point when N is even; evaluated spectrally. */
    double s0 = 0.0;
    for (int k = 0; k < K; ++k) s0 += xh[k];
    st->hist[orc_hist_bin(g->amp * s0, g->u_max)]++;
}

static void stats_finish(orc_stats *st)
{
    if (st->n_grid > 0) {
        double n = (double)st->n_grid;
        double m2 = st->S2 / n, m3 = st->S3 / n, m4 = st->S4 / n;
        st->skewness = m3 / pow(m2, 1.5);
        st->kurtosis = m4 / (m2 * m2);
        st->p_exceed = (double)st->n_exceed / n;
    }
}

/*
 * The rejection sampler over proposal indices [i0, i0+n).  For every index:
 * accept[i-i0] (0/1), and optionally log_a / log_u.  Accepted samples are
 * written in increasing index, up to cap rows of x^ (2K doubles) and index.
 * Statistics cover every accepted sample, written or not.
 * Returns the number accepted.
 */
uint64_t orc_sample(const orc_point *p, uint64_t i0, uint64_t n, uint8_t *accept,
                    double *log_a_out, double *log_u_out, double *xhat_out,
                    uint64_t *index_out, uint64_t cap, orc_stats *st, int nthreads)
{
    int K = p->K;
    uint8_t *acc = accept ? accept : (uint8_t *)malloc(n ? n : 1);
    double max_la = -INFINITY;
    uint64_t nviol = 0;
#pragma omp parallel for num_threads(orc_threads(nthreads)) schedule(static) reduction(max : max_la) reduction(+ : nviol)
    for (int64_t q = 0; q < (int64_t)n; ++q) {
        double xh[2 * ORC_KMAX];
        double lu;
        double la = orc_proposal(p, i0 + (uint64_t)q, xh, &lu);
        acc[q] = (uint8_t)(lu < la);
        if (la > max_la) max_la = la;
        if (la > 0.0) nviol++;
        if (log_a_out) log_a_out[q] = la;
        if (log_u_out) log_u_out[q] = lu;
    }
    orc_stats local;
    orc_grid_table g;
    grid_table_init(&g, K, p->N, p->E0);
    stats_init(&local, &g);
    uint64_t nacc = 0;
    double xh[2 * ORC_KMAX];
    for (uint64_t q = 0; q < n; ++q) {
        if (!acc[q]) continue;
        orc_proposal(p, i0 + q, xh, NULL);
        if (nacc < cap) {
            if (xhat_out)
                for (int m = 0; m < 2 * K; ++m) xhat_out[nacc * 2 * K + m] = xh[m];
            if (index_out) index_out[nacc] = i0 + q;
            local.n_written++;
        }
        stats_add_sample(&local, &g, xh, i0 + q);
        nacc++;
    }
    grid_table_free(&g);
    local.n_proposed = n;
    local.n_accepted = nacc;
    local.n_violations = nviol;
    local.max_log_a = max_la;
    stats_finish(&local);
    if (st) *st = local;
    if (!accept) free(acc);
    return nacc;
}

/*
 * Accepted-count mode: scan proposal indices from 0 in blocks of `block`
 * until n_target samples are accepted or max_proposals are used.  The result
 * is the first n_target accepted samples by index; n_proposed is the index of
 * the last one plus one.
 */
uint64_t orc_sample_until(const orc_point *p, uint64_t n_target, uint64_t max_proposals,
                          double *xhat_out, uint64_t *index_out, uint64_t cap,
                          orc_stats *st, int nthreads)
{
    int K = p->K;
    const uint64_t block = 1u << 16;
    uint8_t *acc = (uint8_t *)malloc(block);
    orc_stats local;
    orc_grid_table g;
    grid_table_init(&g, K, p->N, p->E0);
    stats_init(&local, &g);
    double max_la = -INFINITY;
    uint64_t nacc = 0, last = 0, nviol = 0;
    double xh[2 * ORC_KMAX];
    for (uint64_t base = 0; base < max_proposals && nacc < n_target; base += block) {
        uint64_t nb = max_proposals - base < block ? max_proposals - base : block;
        double *la = (double *)malloc(sizeof(double) * nb);
        orc_sample(p, base, nb, acc, la, NULL, NULL, NULL, 0, NULL, nthreads);
        for (uint64_t q = 0; q < nb && nacc < n_target; ++q) {
            if (la[q] > max_la) max_la = la[q];
            if (la[q] > 0.0) nviol++;
            last = base + q;
            if (!acc[q]) continue;
            orc_proposal(p, base + q, xh, NULL);
            if (nacc < cap) {
                if (xhat_out)
                    for (int m = 0; m < 2 * K; ++m) xhat_out[nacc * 2 * K + m] = xh[m];
                if (index_out) index_out[nacc] = base + q;
                local.n_written++;
            }
            stats_add_sample(&local, &g, xh, base + q);
            nacc++;
        }
        free(la);
    }
    grid_table_free(&g);
    free(acc);
    local.n_proposed = max_proposals ? last + 1 : 0;
    local.n_accepted = nacc;
    local.n_violations = nviol;
    local.max_log_a = max_la;
    stats_finish(&local);
    if (st) *st = local;
    return nacc;
}

/*
 * Per-proposal evaluation of indices [i0, i0+n) for precision studies: H2,
 * H3 (double sum), the grid sums S3 = sum_j u_j^3 and S3abs = sum_j |u_j|^3 of
 * the UNSCALED field u~ = sum_k (x^_k cos k xi_j + x^_{K+k} sin k xi_j) on the
 * N-point grid (direct cos/sin sums), log a and log U.  Any output may be NULL.
 */
void orc_eval_batch(const orc_point *p, uint64_t i0, uint64_t n, double *H2, double *H3,
                    double *S3, double *S3abs, double *log_a, double *log_u, int nthreads)
{
    int K = p->K, N = p->N;
    orc_grid_table g; /* cos(k xi_j), sin(k xi_j) */
    grid_table_init(&g, K, N, p->E0);
#pragma omp parallel for num_threads(orc_threads(nthreads)) schedule(static)
    for (int64_t q = 0; q < (int64_t)n; ++q) {
        double xh[2 * ORC_KMAX];
        double lu;
        double la = orc_proposal(p, i0 + (uint64_t)q, xh, &lu);
        if (H2) H2[q] = orc_H2(K, p->E0, xh);
        if (H3) H3[q] = orc_H3_triad(K, p->E0, xh);
        if (S3 || S3abs) {
            double s3 = 0.0, sa = 0.0;
            for (int j = 0; j < N; ++j) {
                double u = 0.0;
                for (int k = 0; k < K; ++k)
                    u += xh[k] * g.cosv[(size_t)j * K + k] + xh[K + k] * g.sinv[(size_t)j * K + k];
                s3 += u * u * u;
                sa += fabs(u * u * u);
            }
            if (S3) S3[q] = s3;
            if (S3abs) S3abs[q] = sa;
        }
        if (log_a) log_a[q] = la;
        if (log_u) log_u[q] = lu;
    }
    grid_table_free(&g);
}

/* Statistics of an externally supplied set of samples (rows of x^). */
void orc_stats_of(int K, int N, double E0, const double *xhat, uint64_t n, orc_stats *st)
{
    orc_stats local;
    orc_grid_table g;
    grid_table_init(&g, K, N, E0);
    stats_init(&local, &g);
    for (uint64_t s = 0; s < n; ++s) stats_add_sample(&local, &g, xhat + s * 2 * K, s);
    grid_table_free(&g);
    local.n_accepted = n;
    stats_finish(&local);
    *st = local;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

uint64_t orc_mix_sample(const orc_point *p, const orc_mixture *m, uint64_t i0, uint64_t n,
                        uint8_t *accept, double *log_a_out, double *log_u_out, double *xhat_out,
                        uint64_t *index_out, uint64_t cap, int nthreads)
{
    int K = p->K;
#pragma omp parallel for num_threads(orc_threads(nthreads)) schedule(static)
    for (int64_t q = 0; q < (int64_t)n; ++q) {
        double xh[2 * ORC_KMAX], lu;
        double la = orc_mix_proposal(p, m, i0 + (uint64_t)q, xh, &lu);
        accept[q] = (uint8_t)(lu < la);
        if (log_a_out) log_a_out[q] = la;
        if (log_u_out) log_u_out[q] = lu;
    }
    uint64_t nacc = 0;
    double xh[2 * ORC_KMAX];
    for (uint64_t q = 0; q < n; ++q) {
        if (!accept[q]) continue;
        if (nacc < cap) {
            orc_mix_draw(p, m, i0 + q, xh, NULL);
            if (xhat_out)
                for (int c = 0; c < 2 * K; ++c) xhat_out[nacc * 2 * K + c] = xh[c];
            if (index_out) index_out[nacc] = i0 + q;
        }
        nacc++;
    }
    return nacc;
}

/*
 * Sampling-importance resampling with the same proposals, the alternative to
 * the rejection step that the paper names (Sec. I, Sec. IV.B).  For proposal
 * indices [i0, i0+n) in increasing order:
 *   w_i = exp(log a_i) = f/(M g) at proposal i (the importance weight up to
 *         the constant 1/M, the acceptance probability of the rejection step);
 *   W = sum w_i, W2 = sum w_i^2, and the self-normalised grid moments
 *         m_p = sum_i w_i (1/N) sum_j u_ij^p / W, p = 1..4 (u on the N-grid);
 *   C_i = w_0 + ... + w_i; systematic resampling: draw r = 0..m-1 takes the
 *         first proposal with C_i > (u0 + r) W/m.
 * weights[n] (optional), index[m] (proposal indices), sums[8] = {W, W2,
 * max w, m1, m2, m3, m4, number of w > 1}.
 */
void orc_sir(const orc_point *p, uint64_t i0, uint64_t n, uint64_t m, double u0, double *weights,
             uint64_t *index, double *sums, int nthreads)
{
    int K = p->K, N = p->N;
    orc_grid_table g;
    grid_table_init(&g, K, N, p->E0);
    double *w = (double *)malloc(sizeof(double) * (n ? n : 1));
    double *mom = (double *)malloc(sizeof(double) * 4 * (n ? n : 1));
#pragma omp parallel for num_threads(orc_threads(nthreads)) schedule(static)
    for (int64_t q = 0; q < (int64_t)n; ++q) {
        double xh[2 * ORC_KMAX], lu;
        double la = orc_proposal(p, i0 + (uint64_t)q, xh, &lu);
        w[q] = exp(la);
        double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
        for (int j = 0; j < N; ++j) {
            double s = 0.0;
            for (int k = 0; k < K; ++k)
                s += xh[k] * g.cosv[(size_t)j * K + k] + xh[K + k] * g.sinv[(size_t)j * K + k];
            double u = g.amp * s;
            s1 += u;
            s2 += u * u;
            s3 += u * u * u;
            s4 += u * u * u * u;
        }
        mom[4 * q + 0] = s1 / N;
        mom[4 * q + 1] = s2 / N;
        mom[4 * q + 2] = s3 / N;
        mom[4 * q + 3] = s4 / N;
    }
    double W = 0.0, W2 = 0.0, mx = 0.0, M[4] = {0.0, 0.0, 0.0, 0.0};
    uint64_t over = 0;
    for (uint64_t q = 0; q < n; ++q) {
        W += w[q];
        W2 += w[q] * w[q];
        if (w[q] > mx) mx = w[q];
        if (w[q] > 1.0) over++;
        for (int c = 0; c < 4; ++c) M[c] += w[q] * mom[4 * q + c];
        if (weights) weights[q] = w[q];
    }
    /* systematic resampling: walk the cumulative sums once */
    uint64_t q = 0;
    double C = n ? w[0] : 0.0;
    for (uint64_t r = 0; r < m && n; ++r) {
        double pos = (u0 + (double)r) * W / (double)m;
        while (C <= pos && q + 1 < n) {
            q++;
            C += w[q];
        }
        index[r] = i0 + q;
    }
    sums[0] = W;
    sums[1] = W2;
    sums[2] = mx;
    for (int c = 0; c < 4; ++c) sums[3 + c] = W > 0.0 ? M[c] / W : 0.0;
    sums[7] = (double)over;
    free(w);
    free(mom);
    grid_table_free(&g);
}
