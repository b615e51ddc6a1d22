// gfx950 kernels of the TKdV rejection sampler.
//
// Pipeline of one sampling call (all on one stream, no host round trip):
//   k_decide       persistent: per wave, tiles of 32 proposals claimed from a
//                  per-point queue; Philox -> Box-Muller -> scale -> project
//                  -> t, matrix-core synthesis -> sum u^3 -> log a -> decision.
//                  Writes one accept-bit word per tile; proposals within the
//                  decision window go to the FP64 list.
//   k_fixup        FP64 re-decision of the listed proposals (H3 by the double
//                  sum of Sec. IV.A), OR-ed into the accept bitmap.
//   k_seg_count    accepted count per 65536-proposal segment.
//   k_seg_scan     exclusive scan of the segment counts, per point.
//   k_materialize  LDS-staged stream compaction of the accepted bits in
//                  proposal order; regenerates each accepted x^ (same
//                  arithmetic as k_decide), writes it at its rank, and
//                  accumulates FP64 moments, 2-sigma exceedances and the u(0)
//                  histogram from an FP32 matrix-core synthesis.
//   k_finalize     per point, segment partials summed in a fixed order.
//   (mixture)      k_decide_mix and k_fixup_mix take the places of k_decide
//                  and k_fixup for the learned proposal.
#include <hip/hip_runtime.h>

#include "tkdv_device.h"
#include "tkdv_kernels.h"

namespace tkdv {

// ---------------------------------------------------------------------------
// Wave reductions (fixed butterfly order: deterministic)
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_max_f32(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ unsigned long long load_relaxed(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lane 0's value, as a wave-uniform (scalar) value.  The claim loops branch
// on it: a per-lane copy would make their exits divergent for the compiler,
// which may then split a loop so that lanes wait on a lane that has left it.
__device__ __forceinline__ unsigned long long bcast_lane0(unsigned long long v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// Claim kClaimTiles tiles of point C's queue for this wave: every lane issues
// the atomic (lane 0 adds, the others add 0) and lane 0's old value is taken,
// so no lane-divergent region sits next to the loop back-edge (the compiler
// may otherwise thread lanes 1-63 past lane 0's region to the broadcast and
// split the wave).  ~0 when the point's accepted-sample target is met.
__device__ __forceinline__ unsigned long long claim_tiles(const DevPoint &P, DevCounters *C, int lane)
{
    const bool open = P.target == ~0ull || bcast_lane0(load_relaxed(&C->accepted)) < P.target;
    const unsigned long long old =
        atomicAdd(&C->next_tile, (open && lane == 0) ? (unsigned long long)kClaimTiles : 0ull);
    return open ? bcast_lane0(old) : ~0ull;
}

// Per-wave counter update with the same structure: lane 0's (wave-uniform) value.
__device__ __forceinline__ void add_lane0(unsigned long long *ctr, unsigned long long v, int lane)
{
    if (bcast_lane0(v) != 0ull) atomicAdd(ctr, lane == 0 ? v : 0ull);
}

static_assert(kClaimTiles == kWave, "one accept word per lane per claim");

// k_decide's synthesis form: the half-period form (half the matrix work and
// half the tables) where it is faster, the plain product elsewhere
template <int K>
__host__ __device__ constexpr bool decide_half_period() { return K >= 16; }

// k_decide: one staged table (hi or lo)
template <int K, int PREC>
__host__ __device__ constexpr int decide_tab_bytes()
{
    return decide_half_period<K>() ? eo_table_bytes<K, PREC>()
                                   : (PREC == PREC_FP32 ? f32_table_bytes<K>() : bf16_table_bytes<K>());
}
template <int K, int PREC>
__host__ __device__ constexpr int decide_lds_bytes()
{
    return (PREC == PREC_BF16X3 ? 2 : 1) * decide_tab_bytes<K, PREC>();
}

// ---------------------------------------------------------------------------
// k_decide
// ---------------------------------------------------------------------------
// B threads per workgroup sharing one copy of the tables; G tile pairs of the
// half-period synthesis with their accumulators live together (a tile variant
// the sweep's autotuner chooses among; G divides the K/16 tile pairs).
template <int K, int PREC, int PROP, int B = decide_block(K), int G = 1>
__global__ void __launch_bounds__(B) k_decide(KernelArgs a, const int *plist, int n_plist)
{
    static_assert(K < 16 || (K / 16) % G == 0, "G must divide the tile pairs");
    extern __shared__ __attribute__((aligned(16))) char lds[];
    constexpr int tab = decide_tab_bytes<K, PREC>();
    if constexpr (!decide_half_period<K>()) {
        const uint4 *s0 = reinterpret_cast<const uint4 *>(a.phi_hi);
        uint4 *d = reinterpret_cast<uint4 *>(lds);
        for (int v = threadIdx.x; v < tab / 16; v += B) d[v] = s0[v];
        if constexpr (PREC == PREC_BF16X3) {
            const uint4 *s1 = reinterpret_cast<const uint4 *>(a.phi_lo);
            for (int v = threadIdx.x; v < tab / 16; v += B) d[tab / 16 + v] = s1[v];
        }
    } else {
        stage_eo_tables<K, PREC, B>(lds, a.phi_hi, a.phi_lo);
    }
    __syncthreads();
    const char *lds_hi = lds;
    const char *lds_lo = lds + tab;
    const int lane = threadIdx.x & 63, half = lane >> 5, pl = lane & 31;
    const int gwave = blockIdx.x * (B / kWave) + (threadIdx.x >> 6);
    int cursor = gwave % n_plist;
    int misses = 0;
    while (misses < n_plist) {
        const int p = __builtin_amdgcn_readfirstlane(plist[cursor]);
        const DevPoint &P = a.pts[p];
        DevCounters *C = a.cnt + p;
        const unsigned long long base = claim_tiles(P, C, lane);
        if (base >= P.n_tiles) {
            cursor = (cursor + 1 == n_plist) ? 0 : cursor + 1;
            ++misses;
            continue;
        }
        misses = 0;
        unsigned long long n_acc = 0, n_def = 0;
        unsigned int n_viol = 0;
        float max_la = -INFINITY;
        uint32_t my_word = 0u;  // accept bits of tile `lane` of this claim
        for (int c = 0; c < kClaimTiles; ++c) {
            const unsigned long long tile = base + c;
            if (tile >= P.n_tiles) break;
            const unsigned long long local = tile * kTile + pl;
            const bool valid = local < P.n;
            const uint64_t i = P.i0 + local;
            float x[K];
            float t;
            uint32_t w_acc;
            // x is not projected: the cube sum of u~' = Phi^T x is scaled by |x|^-3
            const float inv = gen_xhat<K, PROP, false>(P, i, half, x, t, w_acc);
            if (a.dbg_xhat && valid) {
#pragma unroll
                for (int j = 0; j < K; ++j) a.dbg_xhat[local * (2 * K) + half * K + j] = x[j] * inv;
            }
            float s3l;
            if constexpr (decide_half_period<K>()) s3l = eo_cube_sum<K, PREC, G>(x, lds_hi, lds_lo, lane);
            else s3l = synth_cube_sum<K, PREC>(x, lds_hi, lds_lo, lane);
            const float s3 = (s3l + xor32(s3l)) * (inv * inv * inv);
            const float la = log_a_f32<PROP>(P, t, s3);
            // ln U < ln a - tau  <=>  U < a e^-tau (accept); within the window: FP64.
            // U = (w + 1/2) 2^-32; a = 2^(la log2 e) underflows to 0 only where U > a e^tau.
            const float U = __builtin_fmaf((float)w_acc, 2.3283064365386963e-10f, 1.1641532182693481e-10f);
            const float alin = __builtin_amdgcn_exp2f(la * 1.4426950408889634f);
            const float lo_edge = alin * P.e_lo, hi_edge = alin * P.e_hi;
            const bool mine = valid && half == 0;
            // above the bound by no more than the fast path's error (0 < log a <= tau):
            // the decision and the check of eq. (M_sup) are left to the FP64 pass
            const bool near_bound = la > 0.0f && la <= P.tau;
            const bool defer = mine && ((U >= lo_edge && U < hi_edge) || near_bound);
            const bool accept = mine && U < lo_edge && !near_bound;
            const unsigned long long bacc = __ballot(accept);
            const unsigned long long bdef = __ballot(defer);
            if (lane == c) my_word = (uint32_t)bacc;
            n_acc += __popcll(bacc);
            if (mine) {
                // window proposals are counted by their FP64 value (k_fixup)
                n_viol += (la > 0.0f && !defer) ? 1u : 0u;
                max_la = fmaxf(max_la, la);
                if (a.dbg_t) {
                    a.dbg_t[local] = t;
                    a.dbg_s3[local] = s3;
                    a.dbg_log_a[local] = la;
                    a.dbg_log_u[local] = log_u_word(w_acc);
                }
            }
            if (bdef) {
                const unsigned long long nd = __popcll(bdef);
                const unsigned long long slot = bcast_lane0(atomicAdd(a.defer_count, lane == 0 ? nd : 0ull));
                if (defer) {
                    const unsigned long long pos = slot + __popcll(bdef & ((1ull << lane) - 1ull));
                    if (pos < a.defer_cap) a.defer_list[pos] = pack_defer(p, i);
                }
                n_def += nd;
            }
        }
        // one coalesced store of the claim's accept words
        if (base + lane < P.n_tiles) a.bitmap[P.bm_off + base + lane] = my_word;
        const unsigned long long viol = wave_sum_u64(n_viol);
        max_la = wave_max_f32(max_la);
        add_lane0(&C->accepted, n_acc, lane);
        add_lane0(&C->violations, viol, lane);
        add_lane0(&C->deferred, n_def, lane);
        if (__builtin_amdgcn_readfirstlane(__float_as_uint(max_la)) != __float_as_uint(-INFINITY))
            atomicMax(&C->max_log_a_key, lane == 0 ? float_key(max_la) : 0u);
    }
}

// ---------------------------------------------------------------------------
// k_decide_mix: the sampler with the learned mixture proposal.  Workgroups
// visit the points in turn (starting at their own index) and stage the
// point's shift tables in LDS next to the synthesis tables; the waves of a
// workgroup claim tiles of that point until its queue is empty.  Per
// proposal, on top of the paper's steps: the component draw, y = (R_j A V)^T X
// for the S shifts on the matrix cores and log q_mix (mix_log_q_f32).
// ---------------------------------------------------------------------------
template <int K, int PREC>
__host__ __device__ constexpr int mix_ytab_lds_bytes()
{
    return PREC == PREC_FP32 ? mix_ytab_f32_bytes<K>() : (PREC == PREC_BF16X3 ? 2 : 1) * mix_ytab_bf16_bytes<K>();
}
// the mixture kernel's synthesis form and its tables (hi and lo) in LDS
template <int K>
__host__ __device__ constexpr bool mix_half_period() { return K >= 16; }
template <int K, int PREC>
__host__ __device__ constexpr int mix_tab_bytes()
{
    return mix_half_period<K>() ? eo_table_bytes<K, PREC>()
                                : (PREC == PREC_FP32 ? f32_table_bytes<K>() : bf16_table_bytes<K>());
}
template <int K, int PREC>
__host__ __device__ constexpr int decide_mix_lds_bytes()
{
    return (PREC == PREC_BF16X3 ? 2 : 1) * mix_tab_bytes<K, PREC>() + mix_ytab_lds_bytes<K, PREC>() +
           mix_rv_bytes<K>();
}

template <int K, int PREC>
__global__ void __launch_bounds__(kMixBlock) k_decide_mix(KernelArgs a, const int *plist, int n_plist)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    constexpr bool EO = mix_half_period<K>();
    constexpr int tab = mix_tab_bytes<K, PREC>();
    constexpr int phi_bytes = (PREC == PREC_BF16X3 ? 2 : 1) * tab;
    constexpr int yb = PREC == PREC_FP32 ? mix_ytab_f32_bytes<K>() : mix_ytab_bf16_bytes<K>();
    constexpr int ytab_bytes = mix_ytab_lds_bytes<K, PREC>();
    constexpr int rv_bytes = mix_rv_bytes<K>();
    static_assert(phi_bytes % 16 == 0 && ytab_bytes % 16 == 0 && rv_bytes % 16 == 0, "16-byte staging");
    if constexpr (EO) {
        stage_eo_tables<K, PREC, kMixBlock>(lds, a.phi_hi, a.phi_lo);
    } else {
        const uint4 *s0 = reinterpret_cast<const uint4 *>(a.phi_hi);
        uint4 *d = reinterpret_cast<uint4 *>(lds);
        for (int v = threadIdx.x; v < tab / 16; v += kMixBlock) d[v] = s0[v];
        if constexpr (PREC == PREC_BF16X3) {
            const uint4 *s1 = reinterpret_cast<const uint4 *>(a.phi_lo);
            for (int v = threadIdx.x; v < tab / 16; v += kMixBlock) d[tab / 16 + v] = s1[v];
        }
    }
    const char *lds_hi = lds;
    const char *lds_lo = lds + tab;
    const char *y_hi = lds + phi_bytes;
    const char *y_lo = lds + phi_bytes + yb;
    const float *rv = reinterpret_cast<const float *>(lds + phi_bytes + ytab_bytes);
    const int lane = threadIdx.x & 63, half = lane >> 5, pl = lane & 31;
    const float Kf = (float)K;
    for (int q = 0; q < n_plist; ++q) {
        const int p = __builtin_amdgcn_readfirstlane(plist[(blockIdx.x + q) % n_plist]);
        const DevPoint &P = a.pts[p];
        const DevMix &M = a.mix[p];
        DevCounters *C = a.cnt + p;
        __syncthreads();  // every wave is done with the previous point's tables
        {
            // y tables of the requested arithmetic, then the RV table
            const char *src = a.mix_tab + M.tab_off;
            const uint4 *sy = reinterpret_cast<const uint4 *>(
                src + (PREC == PREC_FP32 ? 2 * mix_ytab_bf16_bytes<K>() : 0));
            const uint4 *srv = reinterpret_cast<const uint4 *>(
                src + 2 * mix_ytab_bf16_bytes<K>() + mix_ytab_f32_bytes<K>());
            uint4 *dy = reinterpret_cast<uint4 *>(lds + phi_bytes);
            uint4 *drv = reinterpret_cast<uint4 *>(lds + phi_bytes + ytab_bytes);
            if constexpr (EO && PREC != PREC_FP32) {  // the parity layout of the split operands
                stage_parity_frags<K, kMixBlock>(dy, sy, 2);
                if constexpr (PREC == PREC_BF16X3) stage_parity_frags<K, kMixBlock>(dy + yb / 16, sy + yb / 16, 2);
            } else {
                for (int v = threadIdx.x; v < ytab_bytes / 16; v += kMixBlock) dy[v] = sy[v];
            }
            for (int v = threadIdx.x; v < rv_bytes / 16; v += kMixBlock) drv[v] = srv[v];
        }
        __syncthreads();
        while (true) {
            const unsigned long long base = claim_tiles(P, C, lane);
            if (base >= P.n_tiles) break;  // scalar branch
            unsigned long long n_acc = 0, n_def = 0;
            unsigned int n_viol = 0;
            float max_la = -INFINITY;
            uint32_t my_word = 0u;
            for (int c = 0; c < kClaimTiles; ++c) {
                const unsigned long long tile = base + c;
                if (tile >= P.n_tiles) break;
                const unsigned long long local = tile * kTile + pl;
                const bool valid = local < P.n;
                const uint64_t i = P.i0 + local;
                float x[K];
                float t, Qa;
                uint32_t w_acc;
                const float inv = gen_x_mix<K, false>(P, M, rv, i, half, x, t, Qa, w_acc);
                if (a.dbg_xhat && valid) {
#pragma unroll
                    for (int j = 0; j < K; ++j) a.dbg_xhat[local * (2 * K) + half * K + j] = x[j] * inv;
                }
                float s3l;
                f32x16 y0, y1;
                if constexpr (EO && PREC == PREC_FP32) {
                    s3l = cube_sum_eo_f32<K, 1>(x, lds_hi, lane);
                    bf16x8 bh[K / 8], bl[K / 8];
                    mix_y<K, PREC>(x, bh, bl, y_hi, y_lo, lane, y0, y1);
                } else if constexpr (EO && PREC == PREC_BF16X3) {
                    constexpr int S = eo_steps<K>();
                    bf16x8 eh[S], el[S], oh[S], ol[S];
                    split_eo<K, PREC>(x, eh, el, oh, ol);
                    s3l = cube_sum_eo_bf16<K, PREC, 1>(eh, el, oh, ol, lds_hi, lds_lo, lane);
                    mix_y_eo<K, PREC>(x, eh, el, oh, ol, y_hi, y_lo, lane, y0, y1);
                } else if constexpr (EO) {  // BF16: hi operands only
                    constexpr int S = eo_steps<K>();
                    bf16x8 eh[S], oh[S];
                    split_eo_hi<K>(x, eh, oh);
                    s3l = cube_sum_eo_bf16<K, PREC, 1>(eh, nullptr, oh, nullptr, lds_hi, lds_lo, lane);
                    mix_y_eo<K, PREC>(x, eh, nullptr, oh, nullptr, y_hi, y_lo, lane, y0, y1);
                } else {
                    bf16x8 bh[K / 8], bl[K / 8];
                    if constexpr (PREC != PREC_FP32) split_bf16<K, PREC>(x, bh, bl);
                    s3l = cube_sum_ops<K, PREC>(x, bh, bl, lds_hi, lds_lo, lane);
                    mix_y<K, PREC>(x, bh, bl, y_hi, y_lo, lane, y0, y1);
                }
                const float s3 = (s3l + xor32(s3l)) * (inv * inv * inv);
                const float lq = mix_log_q_f32(P, M, y0, y1, Qa, inv * inv, t, Kf);
                const float lf = __builtin_fmaf(P.neg_bp_K2, t, P.c3coef * s3);
                const float la = (lf - lq) - P.log_M;
                const float U = __builtin_fmaf((float)w_acc, 2.3283064365386963e-10f, 1.1641532182693481e-10f);
                const float alin = __builtin_amdgcn_exp2f(la * 1.4426950408889634f);
                const float lo_edge = alin * P.e_lo, hi_edge = alin * P.e_hi;
                const bool mine = valid && half == 0;
                // above the bound by no more than the fast path's error (0 < log a <= tau):
                // the decision and the check of eq. (M_sup) are left to the FP64 pass
                const bool near_bound = la > 0.0f && la <= P.tau;
                const bool defer = mine && ((U >= lo_edge && U < hi_edge) || near_bound);
                const bool accept = mine && U < lo_edge && !near_bound;
                const unsigned long long bacc = __ballot(accept);
                const unsigned long long bdef = __ballot(defer);
                if (lane == c) my_word = (uint32_t)bacc;
                n_acc += __popcll(bacc);
                if (mine) {
                    n_viol += (la > 0.0f && !defer) ? 1u : 0u;  // window proposals: k_fixup_mix
                    max_la = fmaxf(max_la, la);
                    if (a.dbg_t) {
                        a.dbg_t[local] = t;
                        a.dbg_s3[local] = s3;
                        a.dbg_log_a[local] = la;
                        a.dbg_log_u[local] = log_u_word(w_acc);
                    }
                }
                if (bdef) {
                    const unsigned long long nd = __popcll(bdef);
                    const unsigned long long slot =
                        bcast_lane0(atomicAdd(a.defer_count, lane == 0 ? nd : 0ull));
                    if (defer) {
                        const unsigned long long pos = slot + __popcll(bdef & ((1ull << lane) - 1ull));
                        if (pos < a.defer_cap) a.defer_list[pos] = pack_defer(p, i);
                    }
                    n_def += nd;
                }
            }
            if (base + lane < P.n_tiles) a.bitmap[P.bm_off + base + lane] = my_word;
            const unsigned long long viol = wave_sum_u64(n_viol);
            max_la = wave_max_f32(max_la);
            add_lane0(&C->accepted, n_acc, lane);
            add_lane0(&C->violations, viol, lane);
            add_lane0(&C->deferred, n_def, lane);
            if (__builtin_amdgcn_readfirstlane(__float_as_uint(max_la)) != __float_as_uint(-INFINITY))
                atomicMax(&C->max_log_a_key, lane == 0 ? float_key(max_la) : 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// k_fixup: FP64 evaluation of listed proposals, as the paper states it:
// normals from the same words, X = Sigma^{1/2} z, X^ = X/|X|, H2 by Parseval,
// H3 by the double sum, log f/(M g) = -beta H + K log(1 + alpha beta' t/K^3) - log M.
// ---------------------------------------------------------------------------
// Normals z (words 0..2K-1 by Box-Muller pairs) and the last Philox block
// (words 2K..2K+3) of proposal i, in FP64.
__device__ uint4 fp64_normals(const DevPoint &P, uint64_t i, double *x)
{
    const int K = P.K;
    const uint32_t c0 = (uint32_t)i, c1 = (uint32_t)(i >> 32);
    const double pi = 3.14159265358979323846;
    for (int b = 0; b < K / 2; ++b) {
        uint4 w = philox4x32_10(c0, c1, P.point_id, (uint32_t)b, P.key0, P.key1);
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
        for (int q = 0; q < 4; q += 2) {
            const double u1 = ((double)ws[q] + 0.5) * 0x1p-32;
            const double u2 = ((double)ws[q + 1] + 0.5) * 0x1p-32;
            const double r = sqrt(-2.0 * log(u1));
            const double th = 2.0 * pi * u2;
            x[4 * b + q] = r * cos(th);
            x[4 * b + q + 1] = r * sin(th);
        }
    }
    return philox4x32_10(c0, c1, P.point_id, (uint32_t)(K / 2), P.key0, P.key1);
}

// Project onto the sphere; returns t = sum k^2 s_k.
__device__ double fp64_project(int K, double *x)
{
    double r2 = 0.0;
    for (int m = 0; m < 2 * K; ++m) r2 += x[m] * x[m];
    const double r = sqrt(r2);
    for (int m = 0; m < 2 * K; ++m) x[m] /= r;
    double t = 0.0;
    for (int k = 1; k <= K; ++k) t += (double)k * k * (x[k - 1] * x[k - 1] + x[K + k - 1] * x[K + k - 1]);
    return t;
}

__device__ double fp64_log_f(const DevPoint &P, const double *x, double t)
{
    return log_f_fp64(P.K, P.E0, P.beta_p, P.c32, x, t);
}

// FP64 evaluation of a listed proposal of the paper's sampler: normals from
// the same words, X = Sigma^{1/2} z, X^ = X/|X|,
// log f/(M g) = log f + K log(1 + alpha beta' t/K^3) - log M.
__device__ void fp64_eval(const DevPoint &P, uint64_t i, double &log_a, double &log_u)
{
    const int K = P.K;
    double x[2 * TKDV_KMAX];
    const uint4 wl = fp64_normals(P, i, x);
    log_u = log(((double)wl.x + 0.5) * 0x1p-32);
    for (int m = 0; m < 2 * K; ++m) x[m] *= P.sig64[m % K];
    const double t = fp64_project(K, x);
    double lr = fp64_log_f(P, x, t);
    if (P.proposal == PROP_SIGMA) lr += K * log1p(P.alpha_star * P.beta_p * t / ((double)K * K * K));
    log_a = lr - P.log_M64;
}

__global__ void __launch_bounds__(kBlock) k_fixup(KernelArgs a)
{
    const unsigned long long cnt = *a.defer_count;
    const unsigned long long n = cnt < a.defer_cap ? cnt : a.defer_cap;
    for (unsigned long long e = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (unsigned long long)gridDim.x * blockDim.x) {
        const unsigned long long v = a.defer_list[e];
        const int p = (int)(v >> 40);
        const uint64_t i = v & ((1ull << 40) - 1ull);
        const DevPoint &P = a.pts[p];
        double la, lu;
        fp64_eval(P, i, la, lu);
        if (lu < la) {
            const uint64_t local = i - P.i0;
            atomicOr(&a.bitmap[P.bm_off + local / 32], 1u << (local % 32));
            atomicAdd(&a.cnt[p].fix_accepted, 1ull);
        }
        if (la > 0.0) {  // f/(M g) > 1 (eq. M_sup broken): counted here for window proposals
            atomicAdd(&a.cnt[p].violations, 1ull);
            atomicMax(&a.cnt[p].max_log_a_key, float_key((float)la));
        }
    }
}

// ---------------------------------------------------------------------------
// k_fixup_mix: FP64 re-decision of listed proposals of the mixture sampler.
// Each half-wave takes one proposal (two per wave), lane l of the half:
//   * the Box-Muller pair l (coordinates 2l, 2l+1) of the draw of gen_x_mix
//     in FP64, the component from the same word, in integers;
//   * mode n = l + 2 of the double sum over triads of H3;
//   * shift j = l of q_net: x^T L0^-1 x of w = R_j^T x^ as e^T A e + |g|^2,
//     g = G^-1 V^T A w, e = w - V g (no cancellation), over all K modes;
// then a half-wave log-sum-exp over the shifts.
// log a = log f - log q_mix - log M.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double half_sum_f64(double v)
{
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double half_max_f64(double v)
{
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ unsigned long long read_lane_u64(unsigned long long v, int l)
{
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
    return ((unsigned long long)hi << 32) | lo;
}

template <int K>
__global__ void __launch_bounds__(kBlock) k_fixup_mix(KernelArgs a)
{
    static_assert(K <= 32 && kMixS == 32, "one lane per Box-Muller pair, triad mode and shift");
    __shared__ double xs[kBlock / kWave][2][2 * K];
    const int lane = threadIdx.x & 63, h = lane >> 5, l = lane & 31;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double *x = xs[wv][h];
    const double pi = 3.14159265358979323846;
    const unsigned long long cnt = *a.defer_count;
    const unsigned long long n = cnt < a.defer_cap ? cnt : a.defer_cap;
    const unsigned long long nw = (unsigned long long)gridDim.x * (kBlock / kWave);
    for (unsigned long long e0 = 2ull * ((unsigned long long)blockIdx.x * (kBlock / kWave) + wv); e0 < n;
         e0 += 2ull * nw) {
        // a second half past the end repeats the first half's proposal; its
        // result is not used
        const bool item = e0 + h < n;
        const unsigned long long v = a.defer_list[item ? e0 + h : e0];
        const int p = (int)(v >> 40);
        const uint64_t i = v & ((1ull << 40) - 1ull);
        const DevPoint &P = a.pts[p];
        const DevMix &M = a.mix[p];
        const uint32_t c0 = (uint32_t)i, c1 = (uint32_t)(i >> 32);
        const uint4 wl = philox4x32_10(c0, c1, P.point_id, (uint32_t)(K / 2), P.key0, P.key1);
        const int comp = wl.y < M.E ? -1 : (int)((wl.y - M.E) / M.B);
        // eta pair of the component (every lane; used when comp >= 0)
        double e0v = 0.0, e1v = 0.0;
        if (comp >= 0) {
            const double r = sqrt(-2.0 * log(((double)wl.z + 0.5) * 0x1p-32));
            const double th = 2.0 * pi * (((double)wl.w + 0.5) * 0x1p-32);
            e0v = r * cos(th);
            e1v = r * sin(th);
        }
        // coordinate m from its normal z
        auto coord = [&](int m, double z) {
            const int k = m % K + 1;
            if (comp < 0) return P.sig64[k - 1] * z;
            const int mi = (k * comp) & (kMixS - 1);
            const double cs = M.cs64[mi], sn = M.sn64[mi];
            const double *vc = M.V64[k - 1], *vs = M.V64[K + k - 1];
            const bool sinb = m >= K;
            const double r0 = sinb ? vs[0] * cs - vc[0] * sn : vc[0] * cs + vs[0] * sn;
            const double r1 = sinb ? vs[1] * cs - vc[1] * sn : vc[1] * cs + vs[1] * sn;
            return M.sqd64[k - 1] * z + r0 * e0v + r1 * e1v;
        };
        double X0 = 0.0, X1 = 0.0;
        if (l < K) {
            const uint4 w = philox4x32_10(c0, c1, P.point_id, (uint32_t)(l / 2), P.key0, P.key1);
            const uint32_t w1 = (l & 1) ? w.z : w.x, w2 = (l & 1) ? w.w : w.y;
            const double r = sqrt(-2.0 * log(((double)w1 + 0.5) * 0x1p-32));
            const double th = 2.0 * pi * (((double)w2 + 0.5) * 0x1p-32);
            X0 = coord(2 * l, r * cos(th));
            X1 = coord(2 * l + 1, r * sin(th));
        }
        const double inv_r = 1.0 / sqrt(half_sum_f64(X0 * X0 + X1 * X1));
        const double x0 = X0 * inv_r, x1 = X1 * inv_r;
        if (l < K) {
            x[2 * l] = x0;
            x[2 * l + 1] = x1;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        double tk = 0.0;
        if (l < K) {
            const double k0 = (2 * l) % K + 1, k1 = (2 * l + 1) % K + 1;
            tk = k0 * k0 * x0 * x0 + k1 * k1 * x1 * x1;
        }
        const double t = half_sum_f64(tk);
        // H3 by the double sum: lane l takes n = l + 2
        double tri = 0.0;
        {
            const int nn = l + 2;
            if (nn <= K) {
                const double s = sqrt(P.E0 / (2.0 * pi));
                double in_re = 0.0, in_im = 0.0;
                for (int kk = 1; kk < nn; ++kk) {
                    const double pr = s * x[kk - 1], pi_ = -s * x[K + kk - 1];
                    const double qr = s * x[nn - kk - 1], qi = -s * x[K + nn - kk - 1];
                    in_re += pr * qr - pi_ * qi;
                    in_im += pr * qi + pi_ * qr;
                }
                tri = (s * x[nn - 1]) * in_re + (-s * x[K + nn - 1]) * in_im;
            }
        }
        const double H3 = 2.0 * pi * half_sum_f64(tri);
        const double lf = -(P.beta_p / (P.E0 * (double)K * K) * (P.E0 * t - P.c32 * H3));
        // q_net: shift j = l
        double y0 = 0.0, y1 = 0.0;
#pragma unroll 4
        for (int k = 1; k <= K; ++k) {
            const int mi = (k * l) & (kMixS - 1);
            const double cs = M.cs64[mi], sn = M.sn64[mi];
            const double xc = x[k - 1], xsn = x[K + k - 1];
            const double wc = xc * cs - xsn * sn, ws = xsn * cs + xc * sn;
            const double ak = M.a64[k - 1];
            y0 += ak * (M.V64[k - 1][0] * wc + M.V64[K + k - 1][0] * ws);
            y1 += ak * (M.V64[k - 1][1] * wc + M.V64[K + k - 1][1] * ws);
        }
        const double g0 = M.gi64[0][0] * y0 + M.gi64[0][1] * y1;
        const double g1 = M.gi64[1][0] * y0 + M.gi64[1][1] * y1;
        double qf = g0 * g0 + g1 * g1;
#pragma unroll 4
        for (int k = 1; k <= K; ++k) {
            const int mi = (k * l) & (kMixS - 1);
            const double cs = M.cs64[mi], sn = M.sn64[mi];
            const double xc = x[k - 1], xsn = x[K + k - 1];
            const double wc = xc * cs - xsn * sn, ws = xsn * cs + xc * sn;
            const double ec = wc - (M.V64[k - 1][0] * g0 + M.V64[k - 1][1] * g1);
            const double es = ws - (M.V64[K + k - 1][0] * g0 + M.V64[K + k - 1][1] * g1);
            qf += M.a64[k - 1] * (ec * ec + es * es);
        }
        const double lj = -K * log(qf);
        const double mx = half_max_f64(lj);
        const double se = half_sum_f64(exp(lj - mx));
        const double lnet = -0.5 * M.logdetL0 + mx + log(se) - log((double)kMixS);
        const double lg = M.lng - K * log1p(P.alpha_star * P.beta_p * t / ((double)K * K * K));
        const double A = M.log_eps + lg, B = M.log_1m_eps + lnet;
        const double hi = A > B ? A : B;
        const double lq = hi + log(exp(A - hi) + exp(B - hi));
        const double log_u = log(((double)wl.x + 0.5) * 0x1p-32);
        const double log_a = lf - lq - P.log_M64;
        // updates of each half in turn, under a wave-uniform condition at a
        // wave-uniform address (lane 0 of the wave carries the value)
        const bool acc = item && log_u < log_a;
        const bool viol = item && log_a > 0.0;  // f/(M q_mix) > 1, counted here for window proposals
        const unsigned long long bm_word = P.bm_off + (i - P.i0) / 32;
        const uint32_t bit = 1u << ((i - P.i0) % 32);
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            if (__builtin_amdgcn_readlane((int)acc, 32 * hh) != 0) {
                const unsigned long long wrd = read_lane_u64(bm_word, 32 * hh);
                const uint32_t b = __builtin_amdgcn_readlane(bit, 32 * hh);
                const int pp = __builtin_amdgcn_readlane(p, 32 * hh);
                atomicOr(&a.bitmap[wrd], lane == 0 ? b : 0u);
                atomicAdd(&a.cnt[pp].fix_accepted, lane == 0 ? 1ull : 0ull);
            }
            if (__builtin_amdgcn_readlane((int)viol, 32 * hh) != 0) {
                const int pp = __builtin_amdgcn_readlane(p, 32 * hh);
                const unsigned int key = __builtin_amdgcn_readlane(float_key((float)log_a), 32 * hh);
                atomicAdd(&a.cnt[pp].violations, lane == 0 ? 1ull : 0ull);
                atomicMax(&a.cnt[pp].max_log_a_key, lane == 0 ? key : 0u);
            }
        }
        // the next proposals overwrite this wave's copies of x^
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------------------
// Segments
// ---------------------------------------------------------------------------
__device__ __forceinline__ int point_of_segment(const DevPoint *pts, int n_points, unsigned long long gs)
{
    int lo = 0, hi = n_points - 1;
    while (lo < hi) {  // last p with seg_off <= gs
        const int mid = (lo + hi + 1) >> 1;
        if (pts[mid].seg_off <= gs) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ unsigned long long processed_words(const DevPoint &P, const DevCounters &C)
{
    const unsigned long long nt = C.next_tile;
    return nt < P.n_tiles ? nt : P.n_tiles;
}

__global__ void __launch_bounds__(kBlock) k_seg_count(KernelArgs a, unsigned long long total_segs,
                                                      unsigned long long *seg_cnt)
{
    __shared__ unsigned long long red[kBlock / kWave];
    if (a.d_total_segs) total_segs = *a.d_total_segs;
    for (unsigned long long gs = blockIdx.x; gs < total_segs; gs += gridDim.x) {
        const int p = point_of_segment(a.pts, a.n_points, gs);
        const DevPoint &P = a.pts[p];
        const unsigned long long nw = processed_words(P, a.cnt[p]);
        const unsigned long long w0 = (gs - P.seg_off) * kSegWords;
        unsigned long long c = 0;
        for (int k = threadIdx.x; k < kSegWords; k += kBlock) {
            const unsigned long long w = w0 + k;
            if (w < nw) c += __popc(a.bitmap[P.bm_off + w]);
        }
        c = wave_sum_u64(c);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long s = 0;
            for (int w = 0; w < kBlock / kWave; ++w) s += red[w];
            seg_cnt[gs] = s;
        }
        __syncthreads();
    }
}

// One block: per point, exclusive scan of its segment counts.
__global__ void __launch_bounds__(1024) k_seg_scan(KernelArgs a, const unsigned long long *seg_cnt,
                                                   unsigned long long *seg_base, PointResult *res)
{
    __shared__ unsigned long long buf[1024];
    for (int p = 0; p < a.n_points; ++p) {
        const DevPoint &P = a.pts[p];
        unsigned long long run = 0;
        for (unsigned long long s0 = 0; s0 < P.n_segs; s0 += 1024) {
            const unsigned long long s = s0 + threadIdx.x;
            const unsigned long long v = s < P.n_segs ? seg_cnt[P.seg_off + s] : 0ull;
            buf[threadIdx.x] = v;
            __syncthreads();
            for (int o = 1; o < 1024; o <<= 1) {  // Hillis-Steele inclusive scan
                const unsigned long long add = threadIdx.x >= (unsigned)o ? buf[threadIdx.x - o] : 0ull;
                __syncthreads();
                buf[threadIdx.x] += add;
                __syncthreads();
            }
            if (s < P.n_segs) seg_base[P.seg_off + s] = run + buf[threadIdx.x] - v;
            run += buf[1023];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            res[p].n_accepted = run;
            res[p].n_processed = processed_words(P, a.cnt[p]) * kTile < P.n
                                     ? processed_words(P, a.cnt[p]) * kTile
                                     : P.n;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// k_materialize: one block per segment, one wave per quarter segment.
// ---------------------------------------------------------------------------
constexpr int kWaveWords = kSegWords / (kBlock / kWave);  // 512 words per wave
constexpr int kGroupWords = kWave;                         // one word per lane per group
constexpr int kQueue = kGroupWords * 32 + kTile;           // one group's offsets + a partial chunk

template <int K>
__host__ __device__ constexpr int materialize_tab_bytes()
{
    // the FP32 table; for K >= 16 its first half (the half-period form)
    return K >= 16 ? eo_table_bytes<K, PREC_FP32>() : f32_table_bytes<K>();
}
template <int K>
__host__ __device__ constexpr int materialize_lds_bytes()
{
    return materialize_tab_bytes<K>() + (kBlock / kWave) * kQueue * 2 + 1024;
}

template <int K, int PROP>
__global__ void __launch_bounds__(kBlock) k_materialize(KernelArgs a, const int *plist, int n_plist,
                                                        unsigned long long total_segs,
                                                        const unsigned long long *seg_cnt,
                                                        const unsigned long long *seg_base,
                                                        SegStats *seg_stats, PointResult *res,
                                                        float *out_xhat, unsigned long long *out_index)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    constexpr int tab = materialize_tab_bytes<K>();
    uint16_t *lists = reinterpret_cast<uint16_t *>(lds + tab);
    unsigned int *hist = reinterpret_cast<unsigned int *>(lds + tab + (kBlock / kWave) * kQueue * 2);
    __shared__ unsigned long long wave_cnt[kBlock / kWave];
    __shared__ double wave_S[kBlock / kWave][4];
    __shared__ unsigned long long wave_ex[kBlock / kWave][3];
    __shared__ unsigned long long wave_peak_idx[kBlock / kWave];
    __shared__ unsigned int wave_peak_key[kBlock / kWave];
    {
        const uint4 *s0 = reinterpret_cast<const uint4 *>(a.phi_hi);
        uint4 *d = reinterpret_cast<uint4 *>(lds);
        for (int v = threadIdx.x; v < tab / 16; v += kBlock) d[v] = s0[v];
    }
    const int lane = threadIdx.x & 63, half = lane >> 5, pl = lane & 31, wv = threadIdx.x >> 6;
    uint16_t *mylist = lists + wv * kQueue;
    if (a.d_total_segs) total_segs = *a.d_total_segs;
    __syncthreads();
    for (unsigned long long gs = blockIdx.x; gs < total_segs; gs += gridDim.x) {
        const int p = point_of_segment(a.pts, a.n_points, gs);
        const DevPoint &P = a.pts[p];
        bool mine_k = P.K == K && P.proposal == PROP;
        const unsigned long long limit = P.target;  // ranks >= target are not part of the result
        if (!mine_k || seg_cnt[gs] == 0 || seg_base[gs] >= limit) continue;  // block-uniform
        for (int b = threadIdx.x; b < kNBins; b += kBlock) hist[b] = 0u;
        const unsigned long long nw = processed_words(P, a.cnt[p]);
        const unsigned long long seg_w0 = (gs - P.seg_off) * kSegWords;
        const unsigned long long w_first = seg_w0 + (unsigned long long)wv * kWaveWords;
        // this wave's accepted count -> rank base
        unsigned long long c = 0;
        for (int k = lane; k < kWaveWords; k += kWave) {
            const unsigned long long w = w_first + k;
            if (w < nw) c += __popc(a.bitmap[P.bm_off + w]);
        }
        c = wave_sum_u64(c);
        if (lane == 0) wave_cnt[wv] = c;
        __syncthreads();
        unsigned long long rank = seg_base[gs];
        for (int w = 0; w < wv; ++w) rank += wave_cnt[w];
        double S1 = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0;
        unsigned long long n_ex = 0, n_ex4 = 0, n_max4 = 0, peak_idx = ~0ull;
        unsigned int peak_key = 0u;
        // accepted offsets (proposals from the wave's first word) queue up in
        // index order; full chunks are regenerated, the last group flushes
        int queued = 0;
        for (int g = 0; g < kWaveWords / kGroupWords; ++g) {
            const unsigned long long w = w_first + (unsigned long long)g * kGroupWords + lane;
            const uint32_t word = w < nw ? a.bitmap[P.bm_off + w] : 0u;
            const int cntw = __popc(word);
            // inclusive prefix over lanes
            int incl = cntw;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int up = __shfl_up(incl, o, 64);
                if (lane >= o) incl += up;
            }
            const int total = __shfl(incl, 63, 64);
            int pos = queued + incl - cntw;
            uint32_t m = word;
            while (m) {
                const int bit = __ffs(m) - 1;
                m &= m - 1;
                mylist[pos++] = (uint16_t)((g * kGroupWords + lane) * 32 + bit);
            }
            queued += total;
            const int upto = g + 1 == kWaveWords / kGroupWords ? queued : queued & ~(kTile - 1);
            if (upto == 0) continue;
            // the list is written and read by lanes of this wave only
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (int c0 = 0; c0 < upto; c0 += kTile) {
                const bool in_chunk = c0 + pl < upto;
                const int off = in_chunk ? (int)mylist[c0 + pl] : 0;
                const unsigned long long local = w_first * kTile + (unsigned long long)off;
                const uint64_t i = P.i0 + local;
                const unsigned long long r = rank + c0 + pl;
                const bool valid = in_chunk && r < limit;
                float x[K];
                float t;
                uint32_t w_acc;
                if constexpr (PROP == PROP_MIXTURE) {
                    const DevMix &M = a.mix[p];
                    const float *rvg = reinterpret_cast<const float *>(
                        a.mix_tab + M.tab_off + 2 * mix_ytab_bf16_bytes<K>() + mix_ytab_f32_bytes<K>());
                    float Qa;
                    gen_x_mix<K, true>(P, M, rvg, i, half, x, t, Qa, w_acc);
                } else {
                    gen_xhat<K, PROP, true>(P, i, half, x, t, w_acc);
                }
                if (valid && r < P.capacity) {
                    if (out_xhat) {
                        float *row = out_xhat + (P.out_off + r) * P.row_stride + half * K;
#pragma unroll
                        for (int j = 0; j < K; ++j) row[j] = x[j];
                    }
                    if (out_index && half == 0) out_index[P.out_off + r] = i;
                }
                if (valid && half == 0 && r + 1 == limit) a.cnt[p].last_index = i;
                // statistics on the grid: u = sqrt(2 E0/pi) u~, u~ from FP32 products
                // (K >= 16: the half-period form, u~ = E + O and E - O on the two halves)
                const float4 *ftab = reinterpret_cast<const float4 *>(lds);
                float umax = -INFINITY;  // the largest of this lane's grid values of the proposal
                auto fold = [&](float uf) {
                    const double u = P.amp * (double)uf;
                    const double u2 = u * u;
                    S1 += u;
                    S2 += u2;
                    S3 += u2 * u;
                    S4 += u2 * u2;
                    n_ex += uf > kTwoSigmaT ? 1ull : 0ull;    // u > 2 sqrt(E0/pi)
                    n_ex4 += uf > kFourSigmaT ? 1ull : 0ull;  // u > 4 sqrt(E0/pi)
                    umax = fmaxf(umax, uf);
                };
                if constexpr (K >= 16) {
#pragma unroll
                    for (int tp = 0; tp < K / 16; ++tp) {
                        f32x16 ce = {}, co = {};
#pragma unroll
                        for (int q = 0; q < K / 4; ++q) {
                            // entries 0..3: modes 4q+1 (odd), 4q+2 (even), 4q+3 (odd), 4q+4 (even)
                            const float4 av = ftab[(tp * (K / 4) + q) * kWave + lane];
                            co = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, x[4 * q + 0], co, 0, 0, 0);
                            ce = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, x[4 * q + 1], ce, 0, 0, 0);
                            co = __builtin_amdgcn_mfma_f32_32x32x2f32(av.z, x[4 * q + 2], co, 0, 0, 0);
                            ce = __builtin_amdgcn_mfma_f32_32x32x2f32(av.w, x[4 * q + 3], ce, 0, 0, 0);
                        }
                        if (valid) {
#pragma unroll
                            for (int v = 0; v < 16; ++v) {
                                fold(ce[v] + co[v]);
                                fold(ce[v] - co[v]);
                            }
                        }
                    }
                } else {
#pragma unroll
                    for (int tt = 0; tt < K / 8; ++tt) {
                        f32x16 acc = {};
#pragma unroll
                        for (int q = 0; q < K / 4; ++q) {
                            const float4 av = ftab[(tt * (K / 4) + q) * kWave + lane];
                            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, x[4 * q + 0], acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, x[4 * q + 1], acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.z, x[4 * q + 2], acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.w, x[4 * q + 3], acc, 0, 0, 0);
                        }
                        if (valid) {
#pragma unroll
                            for (int v = 0; v < 16; ++v) fold(acc[v]);
                        }
                    }
                }
                // the proposal's grid values are split over lanes l and l + 32
                umax = fmaxf(umax, __shfl_xor(umax, 32, 64));
                if (valid && half == 0) {
                    n_max4 += umax > kFourSigmaT ? 1ull : 0ull;
                    peak_merge(peak_key, peak_idx, float_key(umax), i);
                }
                if (valid && half == 0) {
                    // u(0) = sqrt(2 E0/pi) sum_k x^_k; bin of u(0)/u_max = sum_k x^_k / sqrt(K)
                    double s0 = 0.0;
#pragma unroll
                    for (int j = 0; j < K; ++j) s0 += (double)x[j];
                    double posb = (s0 / sqrt((double)K) + 1.0) * (0.5 * kNBins);
                    int bin = (int)floor(posb);
                    bin = bin < 0 ? 0 : (bin > kNBins - 1 ? kNBins - 1 : bin);
                    atomicAdd(&hist[bin], 1u);
                }
            }
            rank += upto;
            // the partial chunk left moves to the front of the queue
            const int left = queued - upto;
            const uint16_t keep = lane < left ? mylist[upto + lane] : (uint16_t)0;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (lane < left) mylist[lane] = keep;
            queued = left;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        S1 = wave_sum_f64(S1);
        S2 = wave_sum_f64(S2);
        S3 = wave_sum_f64(S3);
        S4 = wave_sum_f64(S4);
        n_ex = wave_sum_u64(n_ex);
        n_ex4 = wave_sum_u64(n_ex4);
        n_max4 = wave_sum_u64(n_max4);
        wave_peak(peak_key, peak_idx);
        if (lane == 0) {
            wave_S[wv][0] = S1;
            wave_S[wv][1] = S2;
            wave_S[wv][2] = S3;
            wave_S[wv][3] = S4;
            wave_ex[wv][0] = n_ex;
            wave_ex[wv][1] = n_ex4;
            wave_ex[wv][2] = n_max4;
            wave_peak_key[wv] = peak_key;
            wave_peak_idx[wv] = peak_idx;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            SegStats st = {0.0, 0.0, 0.0, 0.0, 0ull, 0ull, 0ull, 0ull, ~0ull, 0u, 0u};
            for (int w = 0; w < kBlock / kWave; ++w) {
                st.S1 += wave_S[w][0];
                st.S2 += wave_S[w][1];
                st.S3 += wave_S[w][2];
                st.S4 += wave_S[w][3];
                st.n_exceed += wave_ex[w][0];
                st.n_exceed4 += wave_ex[w][1];
                st.n_max4 += wave_ex[w][2];
                peak_merge(st.peak_key, st.peak_index, wave_peak_key[w], wave_peak_idx[w]);
            }
            const unsigned long long sb = seg_base[gs];
            const unsigned long long se = sb + seg_cnt[gs];
            st.n_samples = (se < limit ? se : limit) - sb;
            seg_stats[gs] = st;
        }
        for (int b = threadIdx.x; b < kNBins; b += kBlock)
            if (hist[b]) atomicAdd(&res[p].hist[b], (unsigned long long)hist[b]);
        __syncthreads();
    }
}

// Per point (one workgroup): segment partials summed in a fixed order --
// each thread takes a contiguous run of segments in order, then a fixed
// pairwise tree over the threads -- so the result does not depend on
// scheduling.
__global__ void __launch_bounds__(kBlock) k_finalize(KernelArgs a, const unsigned long long *seg_cnt,
                                                     const unsigned long long *seg_base,
                                                     const SegStats *seg_stats, PointResult *res)
{
    __shared__ double sS[4][kBlock];
    __shared__ unsigned long long sE[3][kBlock], sN[kBlock], sPI[kBlock];
    __shared__ unsigned int sPK[kBlock];
    const int p = blockIdx.x, tid = threadIdx.x;
    const DevPoint &P = a.pts[p];
    const unsigned long long per = (P.n_segs + kBlock - 1) / kBlock;
    const unsigned long long s0 = per * tid, s1 = s0 + per < P.n_segs ? s0 + per : P.n_segs;
    double S1 = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0;
    unsigned long long ex = 0, ex4 = 0, mx4 = 0, ns = 0, pi = ~0ull;
    unsigned int pk = 0u;
    for (unsigned long long s = s0; s < s1; ++s) {
        const unsigned long long gs = P.seg_off + s;
        if (seg_cnt[gs] == 0 || seg_base[gs] >= P.target) continue;
        const SegStats &st = seg_stats[gs];
        S1 += st.S1;
        S2 += st.S2;
        S3 += st.S3;
        S4 += st.S4;
        ex += st.n_exceed;
        ex4 += st.n_exceed4;
        mx4 += st.n_max4;
        ns += st.n_samples;
        peak_merge(pk, pi, st.peak_key, st.peak_index);
    }
    sS[0][tid] = S1;
    sS[1][tid] = S2;
    sS[2][tid] = S3;
    sS[3][tid] = S4;
    sE[0][tid] = ex;
    sE[1][tid] = ex4;
    sE[2][tid] = mx4;
    sN[tid] = ns;
    sPK[tid] = pk;
    sPI[tid] = pi;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (tid < w) {
            for (int q = 0; q < 4; ++q) sS[q][tid] += sS[q][tid + w];
            for (int q = 0; q < 3; ++q) sE[q][tid] += sE[q][tid + w];
            sN[tid] += sN[tid + w];
            unsigned int k0 = sPK[tid];
            unsigned long long i0 = sPI[tid];
            peak_merge(k0, i0, sPK[tid + w], sPI[tid + w]);
            sPK[tid] = k0;
            sPI[tid] = i0;
        }
        __syncthreads();
    }
    if (tid == 0) {
        res[p].S1 = sS[0][0];
        res[p].S2 = sS[1][0];
        res[p].S3 = sS[2][0];
        res[p].S4 = sS[3][0];
        res[p].n_exceed = sE[0][0];
        res[p].n_exceed4 = sE[1][0];
        res[p].n_max4 = sE[2][0];
        res[p].peak_key = sPK[0];
        res[p].peak_index = sPI[0];
        res[p].n_samples = sN[0];
        res[p].n_written = sN[0] < P.capacity ? sN[0] : P.capacity;
    }
}

// ---------------------------------------------------------------------------
// k_window_advance: after one window of a sweep, one workgroup:
//   per point: fold the window's statistics into the running totals, count
//   the accepted samples (the window's target is what was still missing) and
//   mark the point done when its target is met or its index range used up
//   (a done point gets no tiles);
//   then, in point order: the next window of every active point -- its first
//   index, size, remaining target and capacity, output offset, and its place
//   in the window's accept bitmap and segments.  Adaptive windows take the
//   proposals the point still needs at its measured acceptance, times 1.25
//   (four times the proposals so far while it has accepted none), shared out
//   of the bitmap pool in proportion when they do not fit; otherwise every
//   window has the first window's size.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_window_advance(DevPoint *pts, const DevCounters *cnt,
                                                         const PointResult *res, SweepState *sw, int n_points,
                                                         SweepGlobal *G, const unsigned long long *defer_count)
{
    __shared__ double need[1024];
    __shared__ int any_active;
    if (threadIdx.x == 0) any_active = 0;
    __syncthreads();
    for (int p = threadIdx.x; p < n_points; p += blockDim.x) {
        SweepState &S = sw[p];
        DevPoint &P = pts[p];
        if (S.done) continue;
        any_active = 1;
        const PointResult &r = res[p];
        const DevCounters &c = cnt[p];
        S.total.S1 += r.S1;
        S.total.S2 += r.S2;
        S.total.S3 += r.S3;
        S.total.S4 += r.S4;
        S.total.n_exceed += r.n_exceed;
        S.total.n_exceed4 += r.n_exceed4;
        S.total.n_max4 += r.n_max4;
        // windows come in increasing index: a later one replaces the peak only when larger
        if (r.peak_key > S.total.peak_key) {
            S.total.peak_key = r.peak_key;
            S.total.peak_index = r.peak_index;
        }
        for (int b = 0; b < kNBins; ++b) S.total.hist[b] += r.hist[b];
        S.accepted += r.n_samples;
        S.written += r.n_written;
        S.n_fixups += c.deferred;
        S.n_violations += c.violations;
        if (c.max_log_a_key > S.max_log_a_key) S.max_log_a_key = c.max_log_a_key;
        if (S.accepted >= S.target) {
            S.n_proposed = c.last_index - S.i_start + 1;
            S.done = 1;
        } else {
            S.n_proposed += P.n;
            if (P.i0 + P.n >= S.i_end) S.done = 1;
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (any_active) G->windows += 1;
    if (*defer_count > G->defer_cap) G->overflow = 1;
    // sizes of the next windows, in point order
    double sum_need = 0.0;
    for (int p = 0; p < n_points; ++p) {
        const SweepState &S = sw[p];
        const DevPoint &P = pts[p];
        if (S.done) continue;
        const double next_i0 = (double)(P.i0 + P.n), left = (double)S.i_end - next_i0;
        double w = (double)S.window;
        if (G->adaptive) {
            const double used = (double)(P.i0 + P.n - S.i_start);
            const double missing = (double)(S.target - S.accepted);
            w = S.accepted > 0 ? 1.25 * missing * used / (double)S.accepted : 4.0 * used;
            w = w < (double)S.window ? (double)S.window : w;
        }
        w = w > left ? left : w;
        if (p < 1024) need[p] = w;
        sum_need += w;
    }
    const double pool = (double)G->pool_tiles * kTile;
    const double scale = sum_need > pool ? pool / sum_need : 1.0;
    unsigned long long bm = 0, segs = 0, active = 0;
    for (int p = 0; p < n_points; ++p) {
        SweepState &S = sw[p];
        DevPoint &P = pts[p];
        P.bm_off = bm;
        P.seg_off = segs;
        if (S.done) {
            P.n = 0;
            P.n_tiles = 0;
            P.n_segs = 0;
            continue;
        }
        P.i0 += P.n;
        const unsigned long long left = S.i_end - P.i0;
        unsigned long long w = S.window;
        if (G->adaptive && p < 1024) {
            // whole segments (65536 proposals), at least one, within the pool share
            const double share = need[p] * scale;
            const unsigned long long seg = (unsigned long long)kSegWords * kTile;
            w = (unsigned long long)(share / (double)seg) * seg;
            w = w < seg ? seg : w;
        }
        P.n = left < w ? left : w;
        P.n_tiles = (P.n + kTile - 1) / kTile;
        P.n_segs = (P.n_tiles + kSegWords - 1) / kSegWords;
        P.target = S.target - S.accepted;
        P.capacity = S.capacity > S.written ? S.capacity - S.written : 0;
        P.out_off = S.out_off + S.written;
        bm += P.n_tiles;
        segs += P.n_segs;
        ++active;
    }
    G->total_segs = segs;
    G->active = active;
}

hipError_t launch_window_advance(DevPoint *pts, const DevCounters *cnt, const PointResult *res, SweepState *sw,
                                 int n_points, SweepGlobal *G, const unsigned long long *defer_count, hipStream_t st)
{
    hipLaunchKernelGGL(k_window_advance, dim3(1), dim3(1024), 0, st, pts, cnt, res, sw, n_points, G, defer_count);
    return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t *p, unsigned long long n, uint32_t v)
{
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_bits_to_bytes(const uint32_t *bitmap, unsigned long long n, uint8_t *out)
{
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x)
        out[i] = (uint8_t)((bitmap[i / 32] >> (i % 32)) & 1u);
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
template <int K, int PREC, int PROP, int B = decide_block(K), int G = 1>
static hipError_t launch_decide_t(const KernelArgs &a, const int *plist, int n_plist, int n_cu,
                                  unsigned long long total_tiles, hipStream_t st, int *grid_out)
{
    constexpr int lds = decide_lds_bytes<K, PREC>();
    auto kern = k_decide<K, PREC, PROP, B, G>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, B, lds);
    if (e != hipSuccess) return e;
    if (a.blocks_per_cu > 0 && a.blocks_per_cu < per_cu) per_cu = a.blocks_per_cu;
    if (per_cu < 1) per_cu = 1;
    unsigned long long want = (total_tiles + (unsigned long long)(B / kWave) * kClaimTiles - 1) /
                              ((unsigned long long)(B / kWave) * kClaimTiles);
    unsigned long long grid = (unsigned long long)per_cu * n_cu;
    if (want < grid) grid = want;
    if (grid < 1) grid = 1;
    if (grid_out) *grid_out = (int)grid;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(B), lds, st, a, plist, n_plist);
    return hipGetLastError();
}

template <int K>
static hipError_t launch_decide_k(int prec, int prop, const KernelArgs &a, const int *plist, int n_plist,
                                  int n_cu, unsigned long long tiles, hipStream_t st, int *g)
{
#define TKDV_DISPATCH_P(PR, PP) \
    if (prec == PR && prop == PP) return launch_decide_t<K, PR, PP>(a, plist, n_plist, n_cu, tiles, st, g);
    TKDV_DISPATCH_P(PREC_FP32, PROP_UNIFORM)
    TKDV_DISPATCH_P(PREC_FP32, PROP_SIGMA)
    TKDV_DISPATCH_P(PREC_BF16X3, PROP_UNIFORM)
    TKDV_DISPATCH_P(PREC_BF16X3, PROP_SIGMA)
#undef TKDV_DISPATCH_P
    return hipErrorInvalidValue;
}

template <int K, int PREC, int PROP, int B = decide_block(K), int G = 1>
static int decide_blocks_per_cu_t()
{
    constexpr int lds = decide_lds_bytes<K, PREC>();
    auto kern = k_decide<K, PREC, PROP, B, G>;
    if (hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
        return 1;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, B, lds) != hipSuccess) return 1;
    return per_cu < 1 ? 1 : per_cu;
}

// Tile variants of the paper's-proposal decision kernel (BF16x3 products; the
// sweep's autotuner times them).  Variant 0 is the default configuration;
// variants 1..3 at K = 16, 32, 64 (workgroup threads, tile pairs per group):
//   K = 16: (512, 1), (1024, 1), (768, 1)
//   K = 32: (512, 1), (1024, 1), (256, 2)
//   K = 64: variant 0 is the quarter-period kernel (16 proposals per wave,
//           tkdv_quarter.hip, its own tables); 1..3 the half-period k_decide
//           in (512, 1), (1024, 1), (768, 1)
//   K = 128: the quarter-period kernel in workgroups of 512, 768, 1024
// K = 8, and FP32 products, have variant 0 only.
template <int K>
struct DecideVariant;
template <>
struct DecideVariant<16> {
    static constexpr int B[4] = {decide_block(16), 512, 1024, 768}, G[4] = {1, 1, 1, 1};
};
template <>
struct DecideVariant<32> {
    static constexpr int B[4] = {decide_block(32), 512, 1024, 256}, G[4] = {1, 1, 1, 2};
};
template <>
struct DecideVariant<64> {  // B[0]: the quarter-period kernel's workgroup
    static constexpr int B[4] = {decide_block(64), 512, 1024, kHalfPeriod64Block}, G[4] = {1, 1, 1, 1};
};

template <int K, int V>
static hipError_t launch_variant_t(const KernelArgs &a, const int *plist, int n_plist, int n_cu,
                                   unsigned long long tiles, hipStream_t st, int *g)
{
    return launch_decide_t<K, PREC_BF16X3, PROP_SIGMA, DecideVariant<K>::B[V], DecideVariant<K>::G[V]>(
        a, plist, n_plist, n_cu, tiles, st, g);
}
template <int K, int V>
static int variant_blocks_per_cu_t()
{
    return decide_blocks_per_cu_t<K, PREC_BF16X3, PROP_SIGMA, DecideVariant<K>::B[V], DecideVariant<K>::G[V]>();
}

static bool has_variants(int K, int prec, int prop)
{
    return (K == 16 || K == 32 || K == 64) && prec == PREC_BF16X3 && prop == PROP_SIGMA;
}

int decide_n_variants(int K, int prec)
{
    if (prec != PREC_BF16X3) return 1;
    if (K == 128) return decide128_n_variants();
    return has_variants(K, prec, PROP_SIGMA) ? TKDV_DECIDE_VARIANTS : 1;
}

int decide_variant_block(int K, int variant)
{
    if (variant <= 0 || variant >= TKDV_DECIDE_VARIANTS) return decide_block(K);
    switch (K) {
    case 128: return decide128_variant_block(variant);
    case 16: return DecideVariant<16>::B[variant];
    case 32: return DecideVariant<32>::B[variant];
    case 64: return DecideVariant<64>::B[variant];
    default: return decide_block(K);
    }
}

hipError_t launch_decide_variant(int K, int prec, int prop, int variant, const KernelArgs &a, const int *plist,
                                 int n_plist, int n_cu, unsigned long long tiles, hipStream_t st, int *grid_out)
{
    if (K == 128 && prec == PREC_BF16X3 && prop == PROP_SIGMA && variant > 0 && variant < decide128_n_variants())
        return launch_decide128_variant(variant, a, plist, n_plist, n_cu, tiles, st, grid_out);
    if (variant <= 0 || variant >= TKDV_DECIDE_VARIANTS || !has_variants(K, prec, prop))
        return launch_decide(K, prec, prop, a, plist, n_plist, n_cu, tiles, st, grid_out);
#define TKDV_DISPATCH_V(KK)                                                                          \
    if (K == KK) {                                                                                  \
        if (variant == 1) return launch_variant_t<KK, 1>(a, plist, n_plist, n_cu, tiles, st, grid_out); \
        if (variant == 2) return launch_variant_t<KK, 2>(a, plist, n_plist, n_cu, tiles, st, grid_out); \
        return launch_variant_t<KK, 3>(a, plist, n_plist, n_cu, tiles, st, grid_out);               \
    }
    TKDV_DISPATCH_V(16) TKDV_DISPATCH_V(32) TKDV_DISPATCH_V(64)
#undef TKDV_DISPATCH_V
    return hipErrorInvalidValue;
}

int decide_variant_max_blocks_per_cu(int K, int prec, int variant)
{
    if (K == 128 && prec == PREC_BF16X3 && variant > 0 && variant < decide128_n_variants())
        return decide128_variant_max_blocks_per_cu(variant);
    if (variant <= 0 || variant >= TKDV_DECIDE_VARIANTS || !has_variants(K, prec, PROP_SIGMA))
        return decide_max_blocks_per_cu(K, prec);
#define TKDV_DISPATCH_W(KK)                                             \
    if (K == KK) {                                                     \
        if (variant == 1) return variant_blocks_per_cu_t<KK, 1>();      \
        if (variant == 2) return variant_blocks_per_cu_t<KK, 2>();      \
        return variant_blocks_per_cu_t<KK, 3>();                        \
    }
    TKDV_DISPATCH_W(16) TKDV_DISPATCH_W(32) TKDV_DISPATCH_W(64)
#undef TKDV_DISPATCH_W
    return 1;
}

int decide_max_blocks_per_cu(int K, int prec)
{
#define TKDV_DISPATCH_O(KK, PR) \
    if (K == KK && prec == PR) return decide_blocks_per_cu_t<KK, PR, PROP_SIGMA>();
    TKDV_DISPATCH_O(8, PREC_FP32) TKDV_DISPATCH_O(8, PREC_BF16X3)
    TKDV_DISPATCH_O(16, PREC_FP32) TKDV_DISPATCH_O(16, PREC_BF16X3)
    TKDV_DISPATCH_O(32, PREC_FP32) TKDV_DISPATCH_O(32, PREC_BF16X3)
#undef TKDV_DISPATCH_O
    if (K == 64) return decide_quarter64_max_blocks_per_cu(prec);
    if (K == 128) return decide128_max_blocks_per_cu(prec);
    return 1;
}

hipError_t launch_decide(int K, int prec, int prop, const KernelArgs &a, const int *plist, int n_plist,
                         int n_cu, unsigned long long tiles, hipStream_t st, int *grid_out)
{
    switch (K) {
    case 8: return launch_decide_k<8>(prec, prop, a, plist, n_plist, n_cu, tiles, st, grid_out);
    case 16: return launch_decide_k<16>(prec, prop, a, plist, n_plist, n_cu, tiles, st, grid_out);
    case 32: return launch_decide_k<32>(prec, prop, a, plist, n_plist, n_cu, tiles, st, grid_out);
    case 64: return launch_decide_quarter64(prec, prop, a, plist, n_plist, n_cu, tiles, st, grid_out);
    case 128: return launch_decide128(prec, prop, a, plist, n_plist, n_cu, tiles, st, grid_out);
    default: return hipErrorInvalidValue;
    }
}

template <int K, int PREC>
static hipError_t launch_decide_mix_t(const KernelArgs &a, const int *plist, int n_plist, int n_cu,
                                      unsigned long long total_tiles, hipStream_t st, int *grid_out)
{
    constexpr int lds = decide_mix_lds_bytes<K, PREC>();
    auto kern = k_decide_mix<K, PREC>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kMixBlock, lds);
    if (e != hipSuccess) return e;
    if (a.blocks_per_cu > 0 && a.blocks_per_cu < per_cu) per_cu = a.blocks_per_cu;
    if (per_cu < 1) per_cu = 1;
    unsigned long long want = (total_tiles + (unsigned long long)(kMixBlock / kWave) * kClaimTiles - 1) /
                              ((unsigned long long)(kMixBlock / kWave) * kClaimTiles);
    unsigned long long grid = (unsigned long long)per_cu * n_cu;
    if (want < grid) grid = want;
    if (grid < 1) grid = 1;
    if (grid_out) *grid_out = (int)grid;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kMixBlock), lds, st, a, plist, n_plist);
    return hipGetLastError();
}

hipError_t launch_decide_mix(int K, int prec, const KernelArgs &a, const int *plist, int n_plist, int n_cu,
                             unsigned long long tiles, hipStream_t st, int *grid_out)
{
#define TKDV_DISPATCH_X(KK, PR) \
    if (K == KK && prec == PR) return launch_decide_mix_t<KK, PR>(a, plist, n_plist, n_cu, tiles, st, grid_out);
    TKDV_DISPATCH_X(8, PREC_FP32) TKDV_DISPATCH_X(8, PREC_BF16X3)
    TKDV_DISPATCH_X(16, PREC_FP32) TKDV_DISPATCH_X(16, PREC_BF16X3)
    TKDV_DISPATCH_X(32, PREC_FP32) TKDV_DISPATCH_X(32, PREC_BF16X3)
#undef TKDV_DISPATCH_X
    return hipErrorInvalidValue;
}

hipError_t launch_fixup_mix(int K, const KernelArgs &a, int n_cu, hipStream_t st)
{
    const dim3 g(8 * n_cu), b(kBlock);
    switch (K) {
    case 8: hipLaunchKernelGGL(k_fixup_mix<8>, g, b, 0, st, a); break;
    case 16: hipLaunchKernelGGL(k_fixup_mix<16>, g, b, 0, st, a); break;
    case 32: hipLaunchKernelGGL(k_fixup_mix<32>, g, b, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fixup(const KernelArgs &a, int n_cu, hipStream_t st)
{
    hipLaunchKernelGGL(k_fixup, dim3(4 * n_cu), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_segments(const KernelArgs &a, unsigned long long total_segs, unsigned long long *seg_cnt,
                           unsigned long long *seg_base, PointResult *res, int n_cu, hipStream_t st)
{
    unsigned long long g = total_segs < (unsigned long long)(32 * n_cu) ? total_segs : 32ull * n_cu;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_seg_count, dim3((unsigned)g), dim3(kBlock), 0, st, a, total_segs, seg_cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_seg_scan, dim3(1), dim3(1024), 0, st, a, seg_cnt, seg_base, res);
    return hipGetLastError();
}

template <int K, int PROP>
static hipError_t launch_materialize_t(const KernelArgs &a, const int *plist, int n_plist,
                                       unsigned long long total_segs, const unsigned long long *seg_cnt,
                                       const unsigned long long *seg_base, SegStats *seg_stats,
                                       PointResult *res, float *out_xhat, unsigned long long *out_index,
                                       int n_cu, hipStream_t st)
{
    constexpr int lds = materialize_lds_bytes<K>();
    auto kern = k_materialize<K, PROP>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    unsigned long long g = total_segs < (unsigned long long)(8 * n_cu) ? total_segs : 8ull * n_cu;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)g), dim3(kBlock), lds, st, a, plist, n_plist, total_segs,
                       seg_cnt, seg_base, seg_stats, res, out_xhat, out_index);
    return hipGetLastError();
}

hipError_t launch_materialize(int K, int prop, const KernelArgs &a, const int *plist, int n_plist,
                              unsigned long long total_segs, const unsigned long long *seg_cnt,
                              const unsigned long long *seg_base, SegStats *seg_stats, PointResult *res,
                              float *out_xhat, unsigned long long *out_index, int n_cu, hipStream_t st)
{
    if (K == 64 || K == 128)
        return launch_materialize_quarter(K, prop, a, total_segs, seg_cnt, seg_base, seg_stats, res, out_xhat,
                                          out_index, n_cu, st);
#define TKDV_DISPATCH_M(KK, PP)                                                                          \
    if (K == KK && prop == PP)                                                                           \
        return launch_materialize_t<KK, PP>(a, plist, n_plist, total_segs, seg_cnt, seg_base, seg_stats, \
                                            res, out_xhat, out_index, n_cu, st);
    TKDV_DISPATCH_M(8, PROP_UNIFORM)
    TKDV_DISPATCH_M(8, PROP_SIGMA)
    TKDV_DISPATCH_M(16, PROP_UNIFORM)
    TKDV_DISPATCH_M(16, PROP_SIGMA)
    TKDV_DISPATCH_M(32, PROP_UNIFORM)
    TKDV_DISPATCH_M(32, PROP_SIGMA)
    TKDV_DISPATCH_M(8, PROP_MIXTURE)
    TKDV_DISPATCH_M(16, PROP_MIXTURE)
    TKDV_DISPATCH_M(32, PROP_MIXTURE)
#undef TKDV_DISPATCH_M
    return hipErrorInvalidValue;
}

hipError_t launch_finalize(const KernelArgs &a, const unsigned long long *seg_cnt,
                           const unsigned long long *seg_base, const SegStats *seg_stats, PointResult *res,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_finalize, dim3(a.n_points), dim3(kBlock), 0, st, a, seg_cnt, seg_base, seg_stats, res);
    return hipGetLastError();
}

hipError_t launch_fill_u32(void *p, unsigned long long n_words, uint32_t v, hipStream_t st)
{
    if (n_words == 0) return hipSuccess;
    unsigned long long g = (n_words + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(kBlock), 0, st, (uint32_t *)p, n_words, v);
    return hipGetLastError();
}

hipError_t launch_bits_to_bytes(const uint32_t *bitmap, unsigned long long n, uint8_t *out, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    unsigned long long g = (n + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_bits_to_bytes, dim3((unsigned)g), dim3(kBlock), 0, st, bitmap, n, out);
    return hipGetLastError();
}

}  // namespace tkdv
