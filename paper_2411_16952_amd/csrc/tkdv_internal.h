// Structures shared by the host runtime and the gfx950 kernels of the TKdV
// rejection sampler.  Plain data only; no HIP types in the structs.
#pragma once

#include <stdint.h>

#include "../../include/tkdv.h"

namespace tkdv {

constexpr int kWave = 64;          // CDNA wavefront
constexpr int kTile = 32;          // proposals per wave tile (two lanes per proposal)
constexpr int kBlock = 256;        // threads per workgroup of the sampling kernels
// Workgroup of the default decision kernel of each K: at K <= 32 the
// half-period k_decide; at K = 64 and K = 128 the quarter-period kernel
// (tkdv_quarter.hip): workgroups of 256 threads at K = 64 (32 KB of tables
// with BF16x3, several workgroups per CU), of 768 at K = 128 (128 KB of
// tables, one workgroup of 12 waves per CU, 3 per SIMD).
constexpr int decide_block(int K) { return K == 128 ? 768 : kBlock; }
// The half-period k_decide at K = 64 (a tile variant of the sweep's tuner):
// one copy of its 64 KB of tables served 12 waves, 3 per SIMD (168 registers a
// lane; four waves spill inside the tile loop).
constexpr int kHalfPeriod64Block = 768;
constexpr int kSynthBlock = 512;   // threads per workgroup of the standalone synthesis kernel
constexpr int kClaimTiles = 64;    // tiles claimed per work-queue claim (2048 proposals);
                                   // lane c keeps the accept word of tile c
constexpr int kSegWords = 2048;    // bitmap words per statistics segment (65536 proposals)
constexpr int kNBins = TKDV_NBINS;
constexpr int kMixBlock = 1024;    // threads per workgroup of the mixture sampling kernel
constexpr int kMixS = TKDV_MIX_S;  // xi-shifts of the learned mixture

// Per-point constants, laid out for wave-uniform (scalar) loads; sig is also
// read four floats at a time per lane (K = 128 kernels).
struct alignas(16) DevPoint {
    float sig[TKDV_KMAX];    // proposal standard deviations s_k (1 for the uniform proposal)
    double sig64[TKDV_KMAX]; // the same in FP64 (sqrt of the plan's s_k^2)
    // FP32 fast path: log a = neg_bp_K2 * t + c3coef * S3 + Kf * log1p(g_coef * t) - log_M
    float neg_bp_K2;         // -beta'/K^2
    float c3coef;            // beta' c/(E0 K^2) * (pi/(3N)) * (2 E0/pi)^{3/2}
    float g_coef;            // alpha* beta'/K^3   (Sigma proposal; 0 for uniform)
    float Kf;                // K                  (Sigma proposal; 0 for uniform)
    float log_M;             // log M rounded to FP32
    float tau;               // decision window: |log U - log a| < tau -> FP64 re-decision
    float e_lo, e_hi;        // exp(-tau), exp(tau): the window in terms of U and a
    int32_t K;
    int32_t proposal;
    uint32_t point_id;
    uint32_t key0, key1;     // Philox key = seed
    uint32_t pad0;
    // FP64 re-decision
    double E0, beta_p, c32, alpha_star, log_M64;
    double amp;              // sqrt(2 E0/pi)
    // work description
    uint64_t i0;             // first proposal index
    uint64_t n;              // proposals to cover (upper bound in accepted-count mode)
    uint64_t n_tiles;        // ceil(n / 32)
    uint64_t target;         // accepted-sample target (UINT64_MAX in proposal-count mode)
    uint64_t bm_off;         // first bitmap word of this point
    uint64_t seg_off;        // first statistics segment of this point
    uint64_t n_segs;         // statistics segments of this point
    uint64_t out_off;        // first output row of this point
    uint64_t capacity;       // output rows available to this point
    uint64_t row_stride;     // floats between consecutive output rows
};

// Per-point constants of the learned mixture proposal (see tkdv_mixture).
// Its tables live at tab_off in the mixture table buffer:
//   y tables  B[(q, j)][c] = a_c (R_j V C^T)_{c q} as matrix-core A operands,
//             row tile q (rank index), row j (shift) -- BF16 hi, BF16 lo, FP32;
//             C is the upper Cholesky factor of (I + V^T D^-1 V)^-1 = C^T C, so
//             the products give z_j = C y_j and y_j^T G^-1 y_j = |z_j|^2;
//   RV table  (R_j V)_c for shift j, half h, coordinate k of that half:
//             float2 at ((2 j + h) (2K + 2) + 2 k) floats (rows padded by
//             two floats to spread the shifts over the LDS banks).
struct DevMix {
    float sqd[TKDV_KMAX];    // sqrt(d_k)
    float a[TKDV_KMAX];      // 1/d_k
    float c_net;             // ln(1 - eps) - ln|L0|/2 - ln S
    float c_g;               // ln eps + sum_k ln(1 + alpha beta' k^2/K^3)
    float invB;              // 1/B rounded to FP32
    uint32_t E, B;           // component word: w < E -> g_Sigma, else j = (w - E) div B
    // FP64 re-decision
    double a64[TKDV_KMAX], sqd64[TKDV_KMAX];
    double V64[2 * TKDV_KMAX][TKDV_MIX_R];
    double gi64[TKDV_MIX_R][TKDV_MIX_R];
    double cs64[kMixS], sn64[kMixS];  // cos, sin of 2 pi m/S
    double logdetL0, lng, log_eps, log_1m_eps;
    uint64_t tab_off;        // bytes
    uint64_t pad;
};

template <int K>
constexpr int mix_ytab_bf16_bytes() { return 2 * (K / 8) * kWave * 16; }
template <int K>
constexpr int mix_ytab_f32_bytes() { return 2 * (K / 4) * kWave * 16; }
template <int K>
constexpr int mix_rv_bytes() { return kMixS * 2 * (2 * K + 2) * 4; }
// per point: y hi, y lo, y f32, RV
template <int K>
constexpr int mix_point_bytes()
{
    return 2 * mix_ytab_bf16_bytes<K>() + mix_ytab_f32_bytes<K>() + mix_rv_bytes<K>();
}

// Device-side counters per point (zeroed before every launch sequence).
struct DevCounters {
    unsigned long long next_tile;     // work-queue head (tiles)
    unsigned long long accepted;      // decisions that were definite accepts
    unsigned long long violations;    // proposals with log a > 0
    unsigned long long deferred;      // proposals sent to the FP64 re-decision
    unsigned long long fix_accepted;  // of those, accepted
    unsigned long long last_index;    // accepted-count mode: index of the target-th sample
    unsigned int max_log_a_key;       // order-preserving encoding of the largest log a
    unsigned int pad;
};

// Per-segment partial statistics (FP64 sums in a fixed order).
struct SegStats {
    double S1, S2, S3, S4;
    unsigned long long n_exceed;
    unsigned long long n_samples;
    unsigned long long n_exceed4;   // grid values above 4 sigma
    unsigned long long n_max4;      // samples whose largest grid value is above 4 sigma
    unsigned long long peak_index;  // proposal index of the sample with the largest grid value
    unsigned int peak_key;          // float_key of that value of u~ (0: no sample)
    unsigned int pad;
};

// Per-point result of the finalisation kernel.
struct PointResult {
    double S1, S2, S3, S4;
    unsigned long long n_exceed;
    unsigned long long n_exceed4, n_max4, peak_index;  // as in SegStats
    unsigned int peak_key, pad;
    unsigned long long n_samples;      // accepted samples covered by the statistics
    unsigned long long n_accepted;     // all accepted in the processed range
    unsigned long long n_written;
    unsigned long long n_processed;    // proposals whose decision exists
    unsigned long long hist[kNBins];
};

// Per-point state of a windowed sweep (accepted-count sampling in windows of
// proposals; the device advances it after every window).
struct SweepState {
    uint64_t i_start, i_end;      // proposal indices [i_start, i_end) of the point
    uint64_t window;              // proposals of the first window (of every window when not adaptive)
    uint64_t target;              // accepted samples wanted
    uint64_t capacity, out_off;   // output rows of the point
    uint64_t accepted;            // accepted samples so far (at most target)
    uint64_t written;             // rows written so far
    uint64_t n_proposed;          // proposals consumed (up to the target-th sample)
    uint64_t n_fixups, n_violations;
    uint32_t done, max_log_a_key;
    PointResult total;            // statistics of the accepted samples so far
};

// Shared state of a sweep on the device.
struct SweepGlobal {
    unsigned long long pool_tiles;   // accept-bitmap words available to one window
    unsigned long long total_segs;   // statistics segments of the current window
    unsigned long long active;       // points not done
    unsigned long long windows;      // windows run with at least one point active
    unsigned long long overflow;     // a window's FP64 re-decision list overflowed
    unsigned long long defer_cap;
    int adaptive;                    // 1: size each window from the measured acceptance
    int pad;
};

struct KernelArgs {
    const DevPoint *pts;
    int n_points;
    int blocks_per_cu;     // decide-kernel workgroups per compute unit (0: as many as fit)
    DevCounters *cnt;
    uint32_t *bitmap;
    unsigned long long *defer_list;
    unsigned long long *defer_count;
    unsigned long long defer_cap;
    const void *phi_hi;    // BF16 fragment table (hi), or FP32 fragment table
    const void *phi_lo;    // BF16 fragment table (lo)
    const DevMix *mix;     // per point (learned proposal only)
    const char *mix_tab;   // mixture tables (learned proposal only)
    // optional per-proposal outputs of the evaluation entry point (point 0 only)
    float *dbg_xhat, *dbg_t, *dbg_s3, *dbg_log_a, *dbg_log_u;
    // sweeps: the current window's segment count on the device (the windows
    // change size there); NULL elsewhere (the launch's own count is used)
    const unsigned long long *d_total_segs;
};

}  // namespace tkdv
