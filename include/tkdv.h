/*
 * tkdv.h -- C ABI of the MI355X (gfx950) rejection sampler for the Gibbs
 * measure of the truncated Korteweg-de Vries (TKdV) system on the energy
 * sphere S^{2K-1} (N. J. Moore & B. Foerster, arXiv 2411.16952).
 *
 * What is computed (all references are to that paper):
 *   - the target density f(x^) = Z^-1 exp(-beta H_K[U(x^)]) on S^{2K-1}
 *     w.r.t. the uniform measure mu0 (Sec. II.C), with
 *       beta H_K = beta'/(E0 K^2) (H2 - (C3/C2) H3)            (Sec. IV.A)
 *       H2 = E0 sum_k k^2 (x^_k^2 + x^_{K+k}^2)                 (Sec. III.A)
 *       H3 = (1/6) int u^3 dxi                                  (Sec. II.A);
 *   - the paper's proposal g: X ~ N(0, Sigma), Sigma = diag(s^2, s^2),
 *     s_k^2 = 1/(1 + alpha* beta' k^2/K^3), alpha* the root of F (Sec. III.A),
 *     projected X^ = X/|X|, with density ~ (1 + alpha* beta' t/K^3)^-K,
 *     t = sum k^2 (x^_k^2 + x^_{K+k}^2) (Sec. III.B); or the uniform proposal
 *     mu0 (X ~ N(0, I), Sec. II.C), the paper's baseline;
 *   - the rejection algorithm of Sec. IV.B: accept X^ with probability
 *     f/(M g), M = sup f/g (Sec. IV.A), precomputed once per point.
 *
 * Data layout.  A sample is x^ in R^{2K}, stored as 2K consecutive floats
 * [x^_1..x^_K | x^_{K+1}..x^_{2K}]; the Fourier coefficients are
 * u^_k = sqrt(E0/2pi) (x^_k - i x^_{K+k}) (Sec. II.C) and the surface
 * displacement is u(xi) = sqrt(2 E0/pi) sum_k (x^_k cos k xi + x^_{K+k} sin k xi).
 *
 * Random numbers.  Proposal i of a point with stream (seed, point_id) uses
 * Philox4x32-10 with key (seed_lo, seed_hi) and counters
 * (i_lo, i_hi, point_id, j), j = 0..K/2; its words 0..2K-1 give the 2K
 * Box-Muller normals (words 2m, 2m+1 -> z_2m = r cos 2pi U2,
 * z_2m+1 = r sin 2pi U2, r = sqrt(-2 ln U1), U = (w + 1/2) 2^-32) and word 2K
 * gives the acceptance uniform.  Results are a deterministic function of
 * (point, proposal, plan, seed, point_id, n, precision): independent of the
 * launch configuration and of the stream's other work.
 *
 * Exactness.  The fast path evaluates log a = log f/(M g) in FP32 with the
 * spectral-to-grid synthesis on the matrix cores; every proposal whose
 * |log U - log a| is below a proven bound on the fast path's error is
 * re-decided in FP64 (H3 by the double sum of Sec. IV.A), so every accept
 * decision equals the FP64 decision.
 *
 * Conventions.  All functions return a tkdv_status (0 = TKDV_OK).  Device
 * pointers are caller-owned HIP device allocations; host pointers are plain
 * host memory.  `stream` is a hipStream_t (NULL = the default stream); calls
 * are stream-ordered and return after the host-side statistics are complete.
 * Supported mode counts on the GPU: K in {8, 16, 32, 64, 128}, grid N = 4K
 * (the learned mixture K <= 32).  At K = 128 the grid sum of cubes behind H3
 * is formed on the grid offset by half a step (exact there as well, N >= 3K+1)
 * from a quarter of it: the cos and sin blocks and the even and odd modes are
 * synthesised separately, and the four quadrants follow by symmetry.
 */
#ifndef TKDV_H
#define TKDV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TKDV_KMAX 128
#define TKDV_NBINS 64

typedef enum {
    TKDV_OK = 0,
    TKDV_E_ARG = -1,           /* bad size, pointer, enum, non-finite or out-of-range value    */
    TKDV_E_NO_ALPHA_ROOT = -2, /* F has no root: beta' >= K^2 sum_{k<=K} 1/k^2 (Sec. III.A)   */
    TKDV_E_DEVICE = -3,        /* a HIP call failed; tkdv_last_error() has the text            */
    TKDV_E_CAPACITY = -4,      /* an internal work list overflowed                            */
    TKDV_E_UNSUPPORTED = -5,   /* K not supported on the GPU path, or plain BF16 decisions     */
    TKDV_E_M_VIOLATION = -6    /* a proposal had f/(M g) > 1 and the policy did not repair it */
} tkdv_status;

/*
 * The rejection bound f <= M g must hold on the whole sphere (Sec. IV.A, the
 * definition of M as a supremum); M comes from a numerical search, which
 * bounds the supremum only from below.  Every sampling call counts proposals
 * with log a = log f/(M g) > 0 (n_M_violations; decisions inside the FP64
 * window by their FP64 value) and then acts by the context's policy:
 *   TKDV_MV_RAISE (default): raise log M above the largest log a seen (its
 *     FP32 value, plus half the decision window that bounds that value's
 *     error, plus log 1.02), discard the point's output and run it again from
 *     its first proposal, at most 4 times; the learned mixture then falls back
 *     to the paper's Sigma sampler (planned on the host), the paper's
 *     proposals return TKDV_E_M_VIOLATION.  The statistics report the log M
 *     of the returned samples, the number of raises and the fallback;
 *   TKDV_MV_FAIL: return TKDV_E_M_VIOLATION (outputs are those of the run);
 *   TKDV_MV_COUNT: only count (the samples are then not exact).
 */
typedef enum { TKDV_MV_RAISE = 0, TKDV_MV_FAIL = 1, TKDV_MV_COUNT = 2 } tkdv_violation_policy;

typedef enum { TKDV_PROP_UNIFORM = 0, TKDV_PROP_SIGMA = 1, TKDV_PROP_MIXTURE = 2 } tkdv_proposal;

/*
 * Learned proposal (an extension, not in the paper): the defensive mixture
 *   q_mix = eps g_Sigma + (1 - eps) q_net,   q_net = (1/S) sum_{j<S} ACG_j,
 * of angular central Gaussian densities w.r.t. mu0, exactly normalised:
 *   ACG(x^; L) = |L|^{-1/2} (x^T L^{-1} x^)^{-K};
 * g_Sigma (the paper's proposal, Sec. III.B) is the ACG with L = Sigma.
 * Component j is the base L0 = D + V V^T (D = diag(exp logd_k) on the cos and
 * sin coordinate of mode k, V of rank TKDV_MIX_R) rotated by the xi-shift
 * phi_j = 2 pi j/S: (R x)_k = x_k cos k phi + x_{K+k} sin k phi,
 * (R x)_{K+k} = x_{K+k} cos k phi - x_k sin k phi; the target f is invariant
 * under these shifts.  Since q_mix >= eps g_Sigma, f/q_mix <= M_Sigma/eps.
 * Draw of proposal i: the 2K normals zeta of words 0..2K-1, word 2K the
 * acceptance uniform, word 2K+1 the component word w_c, words 2K+2, 2K+3 a
 * Box-Muller pair eta.  The component is chosen in integers: with
 * E = S floor(eps 2^32/S) and B = (2^32 - E)/S, w_c < E -> X = Sigma^{1/2} zeta,
 * otherwise j = (w_c - E) div B, X = D^{1/2} zeta + (R_j V) eta; x^ = X/|X|.
 * The weight of g_Sigma in every density is therefore E 2^-32 (eps rounded
 * down to a multiple of 2^-27).
 */
#define TKDV_MIX_S 32
#define TKDV_MIX_R 2
typedef struct {
    int32_t K;
    int32_t pad;
    double eps;                            /* weight of g_Sigma, e.g. 0.2                */
    double logd[TKDV_KMAX];                /* log d_k, k = 1..K                          */
    double V[2 * TKDV_KMAX][TKDV_MIX_R];   /* base rank-R factor, rows = coordinates     */
} tkdv_mixture;

/* Arithmetic of the spectral-to-grid synthesis U = X^ Phi on the matrix cores:
 * FP32 products, BF16 products (one term), or BF16 with 3-term split
 * (hi*hi + hi*lo + lo*hi) and FP32 accumulation.  All other per-proposal
 * arithmetic is FP32; the decision window is re-evaluated in FP64.
 * Worst-case error of H3 against the cube-sum scale (pi/3N) sum_j |u_j|^3,
 * measured on 2^21 proposals at K = 64: FP32 below 1e-6, BF16x3 below 1e-5,
 * plain BF16 2.9e-3 (median 2.8e-4).  Plain BF16 therefore misses a 1e-3
 * tolerance on H and is offered by tkdv_synthesize only: every entry point
 * that takes accept decisions returns TKDV_E_UNSUPPORTED for it.             */
typedef enum { TKDV_FP32 = 0, TKDV_BF16 = 1, TKDV_BF16X3 = 2 } tkdv_precision;

typedef enum { TKDV_COUNT_PROPOSALS = 0, TKDV_COUNT_ACCEPTED = 1 } tkdv_count_mode;

/* One parameter point: K modes, energy E0, normalised inverse temperature
 * beta' = E0 C2 K^2 beta (Sec. III.A) and the ratio C3/C2 (Sec. IV.A). */
typedef struct {
    int32_t K;
    uint32_t point_id; /* third Philox counter word: distinct streams per point */
    double E0;
    double beta_p;
    double c32;
    uint64_t seed;     /* Philox key */
} tkdv_point;

/* Per-point precompute, plain data (step 1 of Sec. IV.B). */
typedef struct {
    double alpha_star;          /* root of F (Sigma proposal); 1 for the uniform proposal   */
    double log_M;               /* log of the rejection constant for the unnormalised ratio */
    double log_norm_g;          /* sum_k log(1 + alpha* beta' k^2/K^3)                       */
    double sigma2[TKDV_KMAX];   /* proposal variances s_k^2, k = 1..K                        */
    int32_t N;                  /* synthesis grid, 4K                                        */
    int32_t proposal;           /* tkdv_proposal                                             */
    int32_t M_source;           /* 0 closed form (C3/C2 = 0), 1 host search, 2 GPU search,
                                   3 the mixture's cap log M_Sigma - log_norm_g - log eps */
    int32_t n_optimiser_evals;  /* objective evaluations spent on log_M                      */
} tkdv_plan;

/* Statistics of one point's run (Sec. V: skewness, histograms, 2-sigma; the
 * extremes of Sec. V.D against 4 sigma).  Grid values are u on the N = 4K grid
 * xi_j = -pi + 2 pi j/N of every accepted sample. */
typedef struct {
    uint64_t n_proposed;      /* proposals covered by the statistics                         */
    uint64_t n_accepted;      /* accepted among them                                         */
    uint64_t n_written;       /* samples stored (<= capacity)                                */
    uint64_t n_fp64_fixups;   /* proposals re-decided in FP64                                */
    uint64_t n_M_violations;  /* proposals with log a > 0                                    */
    uint64_t n_exceed_2sigma; /* grid values with u > 2 sqrt(E0/pi) over accepted samples    */
    uint64_t n_grid_values;   /* accepted samples x N                                        */
    double max_log_a;         /* largest log f/(M g) seen (FP32 fast path)                   */
    double S1, S2, S3, S4;    /* sums of u^p over accepted samples x grid, FP64              */
    double skewness;          /* m3 / m2^1.5 (raw moments: each sample has mean 0)           */
    double kurtosis;          /* m4 / m2^2 (Gaussian: 3)                                      */
    double p_exceed_2sigma;   /* n_exceed_2sigma / n_grid_values                             */
    double hist_lo, hist_hi;  /* [-u_max, u_max], u_max = sqrt(2 K E0/pi)                     */
    uint64_t hist_u0[TKDV_NBINS]; /* 64 equal bins of u(0), clamped                          */
    double log_M_used;        /* log M of the returned samples (raised after a violation)    */
    int32_t M_raises;         /* runs repeated with a raised M (TKDV_MV_RAISE)               */
    int32_t fallback;         /* 1: the mixture sampler fell back to the Sigma sampler       */
    uint64_t n_exceed_4sigma; /* grid values with u > 4 sqrt(E0/pi)                          */
    uint64_t n_samples_4sigma;/* accepted samples whose largest grid value is above that     */
    double peak_u;            /* largest grid value over the accepted samples (-inf: none)   */
    uint64_t peak_index;      /* proposal index of the sample attaining it, the lowest among
                                 equal maxima (UINT64_MAX: none)                             */
} tkdv_stats;

/* Device time of the phases of the last tkdv_sample / tkdv_sample_batch /
 * tkdv_eval_proposals call on a context, from HIP events recorded on the
 * call's stream around each phase. */
typedef struct {
    double decide_ms;       /* proposal evaluation and decisions (k_decide launches) */
    double fixup_ms;        /* FP64 re-decision of the window proposals             */
    double segments_ms;     /* accept counts and their scan                         */
    double materialize_ms;  /* ordered output and statistics                        */
    double finalize_ms;     /* per-point reduction                                  */
    double synth_ms;        /* tkdv_synthesize: the synthesis kernel                */
    double total_ms;        /* first to last event                                  */
    int32_t decide_launches;
    int32_t decide_grid;    /* workgroups of the (last) k_decide launch             */
    int32_t decide_block;   /* threads per workgroup                                */
    int32_t windows;        /* tkdv_sample_sweep: windows run                         */
    int32_t graph_launches; /* tkdv_sample_sweep: graph launches (16 windows each)     */
} tkdv_timing;

typedef struct tkdv_ctx tkdv_ctx;

/* Create a context on HIP device `hip_device`: device workspaces, the cos/sin
 * synthesis tables, and the launch configuration.  *out is owned by the
 * caller and released by tkdv_destroy. */
tkdv_status tkdv_create(int hip_device, tkdv_ctx **out);
tkdv_status tkdv_destroy(tkdv_ctx *ctx);

/* Step 1 of Sec. IV.B on the host in FP64: alpha* (Brent on F, Sec. III.A),
 * s_k^2, log_norm_g and log M (closed form for C3/C2 = 0; otherwise
 * Nelder-Mead from the zero-mean Dirichlet kernel of Sec. IV.A plus further
 * starts, then refined by gradient ascent on the sphere).  Needs no device. */
tkdv_status tkdv_plan_point(const tkdv_point *pt, tkdv_proposal proposal, tkdv_plan *out);

/*
 * Step 1 of Sec. IV.B for many points at once, with the rejection constant
 * searched on the GPU (the maximisation of Sec. IV.A).  alpha*, s_k^2 and
 * log_norm_g as tkdv_plan_point; C3/C2 = 0 takes the closed form unless
 * flags has TKDV_PLAN_SEARCH_ALWAYS.  Otherwise log M is the largest value of
 * log f - log g (the unnormalised ratio of tkdv_plan_point; log f alone for
 * the uniform proposal) reached by FP64 L-BFGS ascent on the sphere from
 * n_starts starts per point, one wavefront each: the zero-mean Dirichlet
 * kernel of Sec. IV.A, the single-mode state, and n_starts - 2 directions of
 * independent normal coordinates drawn by Philox4x32-10 with key `seed` and
 * counter (start, point_id, coordinate pair, 0x504C414E), so a point's plan
 * does not depend on the other points of the call.  The value and
 * gradient use the exact N = 4K grid quadrature of H3.  The result is a
 * lower bound on the supremum, like any search (M_source = 2).
 *   n_points >= 0; pts and out: host arrays [n_points]; 1 <= K <= 128 (any
 *   K; points with K > 64 are searched on the host as tkdv_plan_point does,
 *   M_source = 1, their xhat_best row zero);
 *   n_starts in [1, 256]; proposal UNIFORM or SIGMA;
 *   xhat_best: host [n_points][2 TKDV_KMAX] doubles or NULL; row p receives
 *     the maximiser found (first 2K entries, unit norm; zeros where the
 *     closed form was taken);
 *   stream: HIP stream (NULL: the null stream); the call returns after it.
 * Errors: TKDV_E_ARG (bad point, argument or flag), TKDV_E_NO_ALPHA_ROOT (the
 * point's index in tkdv_last_error), TKDV_E_DEVICE.
 */
#define TKDV_PLAN_SEARCH_ALWAYS 1
tkdv_status tkdv_plan_batch(tkdv_ctx *ctx, int32_t n_points, const tkdv_point *pts, tkdv_proposal proposal,
                            int32_t n_starts, uint64_t seed, int32_t flags, tkdv_plan *out, double *xhat_best,
                            void *stream);

/*
 * Extreme wave fields among stored samples (Sec. V: the largest surface
 * displacement among individual samples, against 4 sigma = 4 sqrt(E0/pi)).
 * For each row x^ of d_xhat, u = sqrt(2 E0/pi) Phi^T x^ on the grid
 * xi_j = -pi + 2 pi j/N, N = 4K (FP32 matrix products, at K >= 64 in the
 * quarter-period form: values at xi, -xi, pi - xi, xi - pi from the cos/sin
 * sums over even and odd modes at xi in [0, pi/2)); its maximum u_max and
 * the first grid index j attaining it.  Returns the top_k rows by u_max
 * (descending, ties by lower row index) and the number of rows with
 * u_max > threshold.
 *   K in {8,16,32,64,128}; E0 > 0; d_xhat: device [n][row_stride] floats, 16-byte
 *     aligned, row_stride >= 2K and a multiple of 4 (the sampler's rows);
 *   top_k in [0, TKDV_EXTREMES_MAX_K]; h_rows, h_umax, h_jmax: host arrays
 *     [top_k] (entries beyond n are UINT64_MAX, NaN, -1); h_n_exceed: host;
 *   d_umax [n] floats, d_jmax [n] ints: optional device outputs per row;
 *   stream: HIP stream (NULL: the null stream); the call returns after it.
 * Errors: TKDV_E_ARG, TKDV_E_UNSUPPORTED (K, or more than 65536 rows tied at
 * the k-th largest maximum), TKDV_E_DEVICE.
 */
#define TKDV_EXTREMES_MAX_K 4096
tkdv_status tkdv_extremes(tkdv_ctx *ctx, int32_t K, double E0, const float *d_xhat, uint64_t n, uint64_t row_stride,
                          int32_t top_k, double threshold, uint64_t *h_rows, double *h_umax, int32_t *h_jmax,
                          uint64_t *h_n_exceed, float *d_umax, int32_t *d_jmax, void *stream);

/* Result of tkdv_sir. */
typedef struct {
    uint64_t n;            /* proposals weighted                                          */
    uint64_t m;            /* draws                                                       */
    uint64_t n_over_one;   /* weights above 1 by more than the fast path's error bound    */
                           /* (log w > tau: M is not a bound on f/g there)                */
    uint64_t pad;
    double W;              /* sum of the weights w_i = f/(M g) at proposal i               */
    double W2;             /* sum of w_i^2                                                 */
    double ess;            /* effective sample size W^2/W2                                 */
    double max_w;          /* largest weight                                               */
    double mean, m2, m3, m4;   /* self-normalised grid moments sum_i w_i (1/N) sum_j u_ij^p / W */
    double skewness, kurtosis; /* m3/m2^{3/2}, m4/m2^2                                     */
} tkdv_sir_stats;

/*
 * Sampling-importance resampling with the paper's proposals, the alternative
 * to the rejection step that the paper names (Sec. I, Sec. IV.B).  Proposals
 * 0..n-1 of the point (the sampler's own draws, tkdv_sample) are weighted by
 * w_i = f/(M g) (the fast-path acceptance probability of the rejection step,
 * FP32 with FP32 or BF16x3 synthesis; M cancels in every normalised result).
 * Systematic resampling: draw r = 0..m-1 takes the first proposal whose
 * cumulative weight exceeds (u0 + r) W/m (cumulative sums in FP64, in
 * proposal order, monotone by construction).  The grid moments are over
 * xi_j = -pi + 2 pi j/N; at K = 128 they come from the quarter-period
 * syntheses of the weight, on the grid offset by half a step, where sums of
 * u^p, p <= 3, are the same and u^4's differs by a closed form in the top
 * mode's two coordinates, which is added.
 *   K in {8, 16, 32, 64, 128};
 *   proposal UNIFORM or SIGMA; plan NULL plans internally; 1 <= n < 2^40;
 *   u0 in [0, 1); d_index: device [m] proposal indices (non-decreasing),
 *   required when m > 0; d_xhat: device [m][2K] rows of the drawn proposals
 *   or NULL; d_weight: device [n] weights or NULL; h_stats: host.
 *   stream: HIP stream (NULL: the null stream); the call returns after it.
 * Errors: TKDV_E_ARG, TKDV_E_UNSUPPORTED (BF16 precision, all weights zero
 * with m > 0), TKDV_E_DEVICE.
 */
tkdv_status tkdv_sir(tkdv_ctx *ctx, const tkdv_point *pt, tkdv_proposal proposal, const tkdv_plan *plan, uint64_t n,
                     uint64_t m, double u0, tkdv_precision precision, uint64_t *d_index, float *d_xhat,
                     float *d_weight, tkdv_sir_stats *h_stats, void *stream);

/*
 * Rejection-sample one point (Sec. IV.B steps 2-5) on the GPU.
 *   mode = TKDV_COUNT_PROPOSALS: evaluate proposals 0..n-1;
 *   mode = TKDV_COUNT_ACCEPTED:  continue until n samples are accepted (or
 *          max_proposals are used); the result is the first n accepted by
 *          proposal index.
 * plan: NULL plans internally (tkdv_plan_point).
 * d_xhat [capacity][2K] floats and d_index [capacity] (may be NULL) receive
 * the accepted samples in increasing proposal index; beyond `capacity` they
 * are dropped while the statistics still cover every accepted sample.
 * h_stats (host) is filled on return.
 */
tkdv_status tkdv_sample(tkdv_ctx *ctx, const tkdv_point *pt, tkdv_proposal proposal,
                        const tkdv_plan *plan, uint64_t n, tkdv_count_mode mode,
                        uint64_t max_proposals, tkdv_precision precision,
                        float *d_xhat, uint64_t *d_index, uint64_t capacity,
                        tkdv_stats *h_stats, void *stream);

/*
 * tkdv_sample for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels, outputs and statistics, with every work buffer of the call
 * (accept bitmap, FP64 re-decision list, counters, segment arrays) taken from
 * a fixed array in device memory that the library holds per GPU from its
 * first tkdv_create on that GPU until the process ends (17 MiB); the context
 * has built every K's synthesis tables at creation.  The call allocates
 * nothing, on the device or in pinned host memory.  Limits: plan must not be
 * NULL; proposal UNIFORM or SIGMA; at most 2^26 proposals (n, or
 * max_proposals in accepted-count mode), TKDV_E_ARG beyond; at most 2^20
 * proposals inside the FP64 decision window, TKDV_E_CAPACITY beyond.  All
 * calls on one GPU share the array, so calls that overlap on one GPU (other
 * streams, other threads, other contexts) race; the array keeps the last
 * call's contents, and each call clears what must start at zero.  The
 * violation policy of the context applies (reruns use the same array).
 */
tkdv_status tkdv_sample_noalloc(tkdv_ctx *ctx, const tkdv_point *pt, tkdv_proposal proposal,
                                const tkdv_plan *plan, uint64_t n, tkdv_count_mode mode,
                                uint64_t max_proposals, tkdv_precision precision,
                                float *d_xhat, uint64_t *d_index, uint64_t capacity,
                                tkdv_stats *h_stats, void *stream);

/*
 * Many points in one launch sequence (the points may have different K).
 * pts, plans (may be NULL), n, capacity, out_offset and h_stats are host
 * arrays of length n_points; point p writes rows out_offset[p] ..
 * out_offset[p] + min(capacity[p], accepted) - 1 of d_xhat (row stride
 * 2*TKDV_KMAX floats, so rows of different K share one buffer) and d_index.
 */
tkdv_status tkdv_sample_batch(tkdv_ctx *ctx, int32_t n_points, const tkdv_point *pts,
                              tkdv_proposal proposal, const tkdv_plan *plans,
                              const uint64_t *n, tkdv_count_mode mode, uint64_t max_proposals,
                              tkdv_precision precision, float *d_xhat, uint64_t *d_index,
                              const uint64_t *capacity, const uint64_t *out_offset,
                              tkdv_stats *h_stats, void *stream);

/*
 * Per-proposal evaluation for verification: for proposals i0..i0+n-1 writes
 * (each pointer may be NULL) the fast path's x^ [n][2K], t [n], the grid sum
 * S3 = sum_j u~_j^3 of the unscaled synthesis u~ = X^ Phi [n], log a [n] and
 * log U [n] (FP32), and the final accept decision after the FP64 re-check
 * [n] (0/1 bytes).  Same kernels and arithmetic as tkdv_sample.
 */
tkdv_status tkdv_eval_proposals(tkdv_ctx *ctx, const tkdv_point *pt, tkdv_proposal proposal,
                                const tkdv_plan *plan, uint64_t i0, uint64_t n,
                                tkdv_precision precision, float *d_xhat, float *d_t,
                                float *d_s3, float *d_log_a, float *d_log_u,
                                uint8_t *d_accept, void *stream);

/*
 * The spectral-to-grid synthesis of the fast path on its own, for rows of x^
 * already in device memory: for r < n, with x^ = d_xhat[r][0..2K-1] (the
 * layout above) and the grid xi_j = -pi + 2 pi j/N, N = 4K,
 *   d_s3[r] = sum_j u~_j^3,  u~_j = sum_k (x^_k cos k xi_j + x^_{K+k} sin k xi_j),
 * i.e. H3 = (1/6) int u^3 dxi = (pi/(3N)) (2 E0/pi)^{3/2} d_s3[r] exactly when
 * |x^| = 1 (Sec. II.A; N >= 3K + 1).  The products run on the matrix cores in
 * the requested arithmetic with FP32 accumulation; for K >= 16 the sum is
 * formed from the even- and odd-mode syntheses on half the grid (the other
 * half holds their difference), for K = 128 from a quarter of the grid
 * offset by half a step (the same sum in exact arithmetic, N >= 3K + 1).
 * K in {8, 16, 32, 64, 128}; d_xhat 16-byte aligned; both pointers are
 * device pointers owned by the caller.
 */
tkdv_status tkdv_synthesize(tkdv_ctx *ctx, int32_t K, tkdv_precision precision, const float *d_xhat,
                            uint64_t n, float *d_s3, void *stream);

/* The decision window used for a point: proposals with |log U - log a| below
 * it are re-decided in FP64.  It is twice an upper bound on the fast path's
 * error in log a: the synthesis products of the requested arithmetic and
 * their FP32 accumulation, the error of the FP32 x^ and t, and the FP32
 * rounding of every term of log a and of log U. */
double tkdv_decision_window(const tkdv_point *pt, tkdv_proposal proposal, tkdv_precision precision);

/* Host FP64: log q_net and log q_mix (normalised, w.r.t. mu0) at n points x^
 * (host array [n][2K]); sigma_plan is the Sigma plan of the point (alpha*). */
tkdv_status tkdv_mixture_log_q(const tkdv_point *pt, const tkdv_plan *sigma_plan, const tkdv_mixture *mix,
                               const double *xhat, int32_t n, double *log_q_net, double *log_q_mix);

/* Host FP64: the rejection constant of the mixture proposal, log M_mix = log sup
 * f/q_mix (f unnormalised as in log_M of the Sigma plan), by BFGS ascent on the
 * sphere (analytic gradient) from the zero-mean Dirichlet kernel and its
 * shifts, the Sigma maximiser, n_starts caller points (host [n_starts][2K],
 * may be NULL) and seeded random directions.  The result is raised by
 * log(1 + margin) and capped at log M_Sigma - log_norm_g - log eps (valid since
 * q_mix >= eps g_Sigma).  *out is the Sigma plan with log_M replaced and
 * proposal = TKDV_PROP_MIXTURE; argmax (host [2K], may be NULL) receives the
 * best point found.  M_source: 1, or 3 where the cap applies. */
tkdv_status tkdv_plan_mixture(const tkdv_point *pt, const tkdv_plan *sigma_plan, const tkdv_mixture *mix,
                              const double *starts, int32_t n_starts, double margin, tkdv_plan *out,
                              double *argmax);

/*
 * The same rejection constant for many points at once, searched on the GPU:
 * one wavefront per (point, start) maximises log f - log q_mix by FP64 L-BFGS
 * on the sphere (the search of tkdv_plan_batch with the mixture's log q_mix
 * and its analytic gradient), from the zero-mean Dirichlet kernel, the
 * single-mode state, n_starts - 2 seeded normal directions (key seed, counter
 * (start, point_id, ...)) and n_user caller starts per point.  Margin and cap
 * as tkdv_plan_mixture; M_source 2, or 3 where the cap applies.
 *   pts, sigma_plans, mixes, out: host arrays [n_points]; 1 <= K <= 32;
 *   starts: host [n_points][n_user][2 TKDV_KMAX] (first 2K entries used) or
 *   NULL with n_user = 0; n_starts in [1, 256]; xhat_best: host
 *   [n_points][2 TKDV_KMAX] or NULL; stream: HIP stream; returns after it.
 * Errors: TKDV_E_ARG (a mixture or start that is not finite, K, counts).
 */
tkdv_status tkdv_plan_mixture_batch(tkdv_ctx *ctx, int32_t n_points, const tkdv_point *pts,
                                    const tkdv_plan *sigma_plans, const tkdv_mixture *mixes, const double *starts,
                                    int32_t n_user, int32_t n_starts, uint64_t seed, double margin, tkdv_plan *out,
                                    double *xhat_best, void *stream);

/* tkdv_sample with the learned proposal (plan from tkdv_plan_mixture), same
 * outputs and statistics.  K in {8, 16, 32}: at K = 64 the synthesis and shift
 * tables together exceed the LDS of a compute unit (TKDV_E_UNSUPPORTED).
 * TKDV_E_ARG also when lambda_max(I + V^T D^-1 V) > 1e5 (the FP32 quadratic
 * forms would lose all precision). */
tkdv_status tkdv_sample_mixture(tkdv_ctx *ctx, const tkdv_point *pt, const tkdv_plan *mix_plan,
                                const tkdv_mixture *mix, uint64_t n, tkdv_count_mode mode,
                                uint64_t max_proposals, tkdv_precision precision, float *d_xhat,
                                uint64_t *d_index, uint64_t capacity, tkdv_stats *h_stats, void *stream);

/* tkdv_eval_proposals for the learned proposal: per-proposal x^, t, S3, log a,
 * log U and decisions of proposals [i0, i0 + n) (device arrays as there). */
tkdv_status tkdv_eval_mixture(tkdv_ctx *ctx, const tkdv_point *pt, const tkdv_plan *mix_plan,
                              const tkdv_mixture *mix, uint64_t i0, uint64_t n, tkdv_precision precision,
                              float *d_xhat, float *d_t, float *d_s3, float *d_log_a, float *d_log_u,
                              uint8_t *d_accept, void *stream);

/* Decision window of the mixture sampler for this point, mixture and
 * arithmetic: the window of the paper's proposal plus the error bound of the
 * FP32 log q_mix (input error, y products, rounding, log2/exp2), times 2. */
double tkdv_mixture_window(const tkdv_point *pt, const tkdv_plan *mix_plan, const tkdv_mixture *mix,
                           tkdv_precision precision);

/*
 * Learned proposal, the network (an extension, not in the paper): a
 * multilayer perceptron conditioned on (beta', E0, C3/C2) whose output is the
 * tkdv_mixture of a point, evaluated and trained on the GPU in FP64.
 *   z  = ((beta' - 40)/20, ln E0, (C3/C2) sqrt(E0) beta'/1e4 - 1)
 *   h1 = tanh(W1^T z + b1),  h2 = tanh(W2^T h1 + b2),  o = W3^T h2 + b3
 *   log d_k = log s_k^2 + o_{k-1}          (s_k^2 of the point's Sigma plan)
 *   V = V0 + v_scale * o_{K..5K-1} (row-major [2K][2]), V0 = v_amp/sqrt(K) on
 *       the cos block of column 0 and on the sin block of column 1.
 * Weights, one FP64 array, input-major: W1 [3][H], b1 [H], W2 [H][H], b2 [H],
 * W3 [H][5K], b3 [5K].  Training rows of point p are unit vectors x_s of
 * three kinds: accepted samples of the point (kind 0), points where f/q_mix
 * is large, e.g. the arg max of tkdv_plan_mixture (kind 1), and accepted
 * samples that enter the likelihood term only (kind 2: a large sample set
 * whose soft maximum runs over a subsample, the kind-0 rows).  The loss is
 *   L = sum_p [ T log sum_{s in p, kind 0, 1} exp((log f(x_s) - log q_mix(x_s))/T)
 *               - lambda mean_{s in p, kind 0, 2} log q_net(x_s) ],
 * a soft maximum of the ratio (whose supremum is log M_mix) plus a
 * likelihood term; Adam on the weights.  The mixture densities of the rows
 * and their gradients run as FP64 matrix products (the y products of all
 * shifts at once).  K in {8, 16, 32}.
 */
typedef struct {
    int32_t K;
    int32_t hidden;       /* H, 1..256                                        */
    double eps;           /* weight of g_Sigma in the mixture                 */
    double v_amp;         /* V0 amplitude                                     */
    double v_scale;       /* output scale of V                                */
    double temperature;   /* T > 0                                            */
    double nll_weight;    /* lambda >= 0                                      */
    double lr, beta1, beta2, adam_eps;
    uint64_t seed;        /* initial weights: W1, W2 ~ Glorot uniform, the rest 0 */
} tkdv_learner_cfg;

typedef struct tkdv_learner tkdv_learner;

tkdv_status tkdv_learner_create(tkdv_ctx *ctx, const tkdv_learner_cfg *cfg, tkdv_learner **out);
tkdv_status tkdv_learner_destroy(tkdv_learner *learner);
/* The training points; sigma_plans are their Sigma plans.  Clears the rows. */
tkdv_status tkdv_learner_set_points(tkdv_learner *learner, int32_t n_points, const tkdv_point *pts,
                                    const tkdv_plan *sigma_plans);
/* Append n rows of kind 0, 1 or 2 to point `point`: device FP32 rows
 * (row_stride floats apart, first 2K used) or host FP64 rows [n][2K]; rows
 * are normalised in FP64. */
tkdv_status tkdv_learner_add_rows(tkdv_learner *learner, int32_t point, const float *d_xhat, uint64_t row_stride,
                                  uint64_t n, int32_t kind, void *stream);
tkdv_status tkdv_learner_add_rows_host(tkdv_learner *learner, int32_t point, const double *h_xhat, uint64_t n,
                                       int32_t kind);
/* Append, for each of the n host FP64 rows h_xhat [n][2K] (normalised in
 * FP64), its copies with the field translated by each phase of h_phi
 * [n_phi]: u(xi) -> u(xi + phi), i.e. the (cos, sin) pair of mode k rotated
 * by the angle k phi (f is invariant under these shifts, Sec. II.A-C; the
 * mixture only under multiples of 2 pi/S, so shifted copies of a point where
 * f/q_mix is large are informative rows).  phi = 0 keeps the row itself.
 * Row (r, q) is appended at position r n_phi + q; the rotation runs on the
 * device in FP64.  1 <= n_phi <= 4096, phases finite; TKDV_E_ARG otherwise. */
tkdv_status tkdv_learner_add_shifted_rows(tkdv_learner *learner, int32_t point, const double *h_xhat, uint64_t n,
                                          const double *h_phi, int32_t n_phi, int32_t kind);
/* n_steps Adam steps; h_loss (host [n_points], may be NULL) receives the
 * per-point loss at the weights before the last step. */
tkdv_status tkdv_learner_train(tkdv_learner *learner, int32_t n_steps, double *h_loss, void *stream);
/* One evaluation without update: per-point loss, dL/d(log d_1..K, V row-major)
 * per point (host [n_points][5K]) and dL/dweights (host [n_weights]); each
 * output may be NULL. */
tkdv_status tkdv_learner_gradients(tkdv_learner *learner, double *h_loss, double *h_grad_mix,
                                   double *h_grad_weights, void *stream);
/* The network's mixture at a point (its Sigma plan gives s_k^2). */
tkdv_status tkdv_learner_mixture(tkdv_learner *learner, const tkdv_point *pt, const tkdv_plan *sigma_plan,
                                 tkdv_mixture *out);
int64_t tkdv_learner_n_weights(const tkdv_learner *learner);
tkdv_status tkdv_learner_get_weights(const tkdv_learner *learner, double *h_out, int64_t n);
tkdv_status tkdv_learner_set_weights(tkdv_learner *learner, const double *h_in, int64_t n);

/*
 * Batched sweep (the paper's Sigma proposal): accepted-count sampling of many
 * points of mixed K in windows of proposals.  Launch configuration per
 * (K, arithmetic):
 */
#define TKDV_DECIDE_VARIANTS 4
typedef struct {
    int32_t blocks_per_cu;  /* decide workgroups per compute unit, 0: as many as fit   */
    int32_t use_graph;      /* 1: 16 windows captured in one hipGraph, launched once     */
    uint64_t window;        /* proposals of a point's first window, a multiple of 65536 */
    int32_t variant;        /* tile variant of the decision kernel, 0..3 (BF16x3: at
                               K = 16, 32, 64 workgroup threads x tile pairs per group,
                               or the half- against the quarter-period form; at K = 128
                               0..2, workgroup threads); a variant a K does not have
                               runs its variant 0                                       */
    int32_t adaptive;       /* 1: later windows sized on the device from the measured
                               acceptance; 0: every window `window` proposals           */
} tkdv_launch_cfg;

/* Point p draws proposals i = 0, 1, ... until targets[p] (>= 1) samples are
 * accepted or max_proposals[p] proposals are used (Sec. IV.B's loop, in
 * windows).  One window is one launch sequence over every unfinished point:
 * decisions per K, FP64 re-decision, ordered compaction and statistics, and a
 * device-side advance of every point to its next window.  The first window of
 * a point has `window` proposals; with `adaptive` the device sizes each later
 * one from the point's measured acceptance (1.25 times the proposals still
 * needed, four times those so far while none is accepted), sharing a bitmap
 * pool of up to 2^33 proposals in proportion when they do not fit, so that
 * most points finish in their second window.  16 windows are captured in one
 * hipGraph and launched at once (use_graph; otherwise the same 16 windows are
 * launched directly); the host reads the device state once per 16 windows,
 * and a window without unfinished points does nothing.  Output as in
 * tkdv_sample_batch: the first targets[p] accepted samples by index in rows
 * (out_offset[p] + r) of d_xhat (stride 2 * TKDV_KMAX floats) and d_index, at
 * most capacity[p] rows; stats cover the same samples; n_proposed counts the
 * proposals up to the last of them (or max_proposals[p]).  cfg NULL: the
 * context's configuration of each K (tkdv_set_launch_cfg / tkdv_autotune), by
 * default all workgroups that fit, first windows of 2^26 proposals, variant 0,
 * adaptive; otherwise cfg for every K.  Plans must be Sigma plans (or NULL:
 * planned here). */
tkdv_status tkdv_sample_sweep(tkdv_ctx *ctx, int32_t n_points, const tkdv_point *pts, const tkdv_plan *plans,
                              const uint64_t *targets, const uint64_t *max_proposals, tkdv_precision precision,
                              const tkdv_launch_cfg *cfg, float *d_xhat, uint64_t *d_index,
                              const uint64_t *capacity, const uint64_t *out_offset, tkdv_stats *h_stats,
                              void *stream);

/*
 * Extremes map over parameter space (Sec. V.D: the largest displacements of
 * individual samples against 4 sigma at several (beta', C3/C2); the paper's
 * outlook of ensembles over whole regions of parameter space).  The
 * n_beta x n_c points (K, E0, betas[b], c32s[c]) -- cell b * n_c + c, Philox
 * key `seed`, point_id point_id0 + cell -- are planned on the GPU
 * (tkdv_plan_batch, 16 starts) and sampled with the paper's proposal in one
 * batched sweep (tkdv_sample_sweep, the context's launch configuration and
 * violation policy): n_accepted samples per cell, or max_proposals proposals;
 * no sample is stored.  Each cell gets its plan, counts and moments, and the
 * extremes: the fraction of grid values above 4 sigma, the fraction of
 * samples whose largest grid value is above 4 sigma, and the largest
 * displacement with its sample's proposal index (regenerated by
 * tkdv_eval_proposals with the cell's point and plan).  With n_accepted =
 * 500, peak_u is the 1-in-500 event of Sec. V.D's figures.  A cell without a
 * root alpha* (beta' >= K^2 sum_k 1/k^2, Sec. III.A) gets status
 * TKDV_E_NO_ALPHA_ROOT and is not sampled.
 *   K a sampler K (8, 16, 32, 64, 128); E0 > 0; n_beta, n_c >= 1 with
 *   n_beta n_c <= TKDV_MAP_MAX_CELLS; betas >= 0 and c32s finite: host arrays;
 *   n_accepted >= 1, max_proposals >= 1; precision FP32 or BF16X3;
 *   cells: host [n_beta n_c]; stream: HIP stream (NULL: the null stream),
 *   the call returns after it.
 * Errors: TKDV_E_ARG, TKDV_E_UNSUPPORTED, TKDV_E_DEVICE, TKDV_E_M_VIOLATION
 * (policy TKDV_MV_FAIL).
 */
typedef struct {
    double beta_p, c32;
    double alpha_star, log_M;   /* the cell's plan                                        */
    uint64_t n_proposed, n_accepted;
    double acceptance, skewness, kurtosis;
    double p_exceed_2sigma;     /* grid values above 2 sqrt(E0/pi) / grid values            */
    double p_exceed_4sigma;     /* grid values above 4 sqrt(E0/pi) / grid values            */
    double p_sample_4sigma;     /* samples whose largest grid value is above 4 sigma / n    */
    double peak_u;              /* largest grid value over the samples (-inf: none)         */
    uint64_t peak_index;        /* its sample's proposal index (UINT64_MAX: none)           */
    int32_t status;             /* TKDV_OK, or TKDV_E_NO_ALPHA_ROOT (cell not sampled)      */
    int32_t M_raises;           /* the cell's runs with a raised M                          */
} tkdv_map_cell;
#define TKDV_MAP_MAX_CELLS 4096
tkdv_status tkdv_extremes_map(tkdv_ctx *ctx, int32_t K, double E0, int32_t n_beta, const double *betas,
                              int32_t n_c, const double *c32s, uint64_t seed, uint32_t point_id0,
                              uint64_t n_accepted, uint64_t max_proposals, tkdv_precision precision,
                              tkdv_map_cell *cells, void *stream);

/* The context's launch configuration of the sweep for (K, precision). */
tkdv_status tkdv_set_launch_cfg(tkdv_ctx *ctx, int32_t K, tkdv_precision precision, const tkdv_launch_cfg *cfg);
tkdv_status tkdv_get_launch_cfg(const tkdv_ctx *ctx, int32_t K, tkdv_precision precision, tkdv_launch_cfg *out);

/* Autotuner: times a probe sweep (16 points of this K, beta' in [20, 60],
 * a fixed number of proposals each) for every tile variant of the decision
 * kernel (TKDV_DECIDE_VARIANTS: workgroup size and tile pairs per group, at
 * K = 16, 32, 64 with BF16x3), every blocks_per_cu that fits it, and first
 * windows of 2^24, 2^25 and 2^26 proposals; keeps the fastest (proposals/s),
 * stores it in the context and, when cache_path is not NULL, in a text cache
 * keyed by device, K and precision (a cached entry is used without timing).
 * *out (may be NULL) receives the choice. */
tkdv_status tkdv_autotune(tkdv_ctx *ctx, int32_t K, tkdv_precision precision, const char *cache_path,
                          tkdv_launch_cfg *out);

/* The context's policy for proposals with f/(M g) > 1 (see tkdv_violation_policy). */
tkdv_status tkdv_set_violation_policy(tkdv_ctx *ctx, tkdv_violation_policy policy);

/* Phase timings of the last call on this context (see tkdv_timing). */
tkdv_status tkdv_get_timing(const tkdv_ctx *ctx, tkdv_timing *out);

const char *tkdv_status_str(tkdv_status s);
/* Text of the last error on this context (or of the last context-less call). */
const char *tkdv_last_error(const tkdv_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* TKDV_H */
