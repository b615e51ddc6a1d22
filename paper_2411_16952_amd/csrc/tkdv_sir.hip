// Sampling-importance resampling (SIR) with the paper's proposals, the
// alternative to the rejection step that the paper names (Sec. I, Sec. IV.B).
//
//   k_sir_weights   per proposal the fast-path log a of the rejection sampler
//                   (the same draw, synthesis and arithmetic as k_decide) and
//                   the weight w = exp(log a) = f/(M g); per tile the FP64
//                   sum of the weights; per wave FP64 partials of sum w^2,
//                   max w, sum w S_p (S_p = sum_j u~_j^p, p = 1..4) and the
//                   count of w > 1;
//   k_sir_scan_*    exclusive prefix of the tile sums, in a fixed order
//                   (chunks of kSirChunk tiles, then the chunk sums);
//   k_sir_resample  systematic resampling: draw r takes the proposal whose
//                   cumulative-weight interval holds (u0 + r) W/m.  Proposal
//                   i gets draws [A(C_{i-1}), A(C_i)), A(c) = ceil(c m/W - u0)
//                   clamped to the tile's range [A(off_t), A(off_t+1)), so the
//                   m draws are partitioned exactly; each lane writes its own
//                   proposal's draws (no atomics), and the rows of x^ when asked.
// At K = 128 the weights and the rows come from the quarter-period kernels'
// draw and synthesis (k_sir_weights_q, k_sir_resample_q: tkdv_quarter.h), so
// that w = f/(M g) is the decision kernel's and the rows are the sampler's.
#include "tkdv_device.h"
#include "tkdv_quarter.h"
#include "tkdv_sir.h"

namespace tkdv {
namespace {

__device__ __forceinline__ double sum64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double max64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// One staged synthesis table (hi or lo): the half-period form for K >= 16,
// the plain table at K = 8.
template <int K, int PREC>
__host__ __device__ constexpr int sir_tab_bytes()
{
    return K >= 16 ? eo_table_bytes<K, PREC>() : (PREC == PREC_FP32 ? f32_table_bytes<K>() : bf16_table_bytes<K>());
}

// The power sums of the half-period form: with u~ = E + O on grid tile t and
// E - O on tile t + T/2, per pair of grid values
//   sum u~ = 2E, sum u~^2 = 2(E^2 + O^2), sum u~^3 = 2E(E^2 + 3 O^2),
//   sum u~^4 = 2((E^2 + O^2)^2 + 4 E^2 O^2);
// the factor 2 is applied at the end.
__device__ __forceinline__ void pair_power_sums(const f32x16 &ce, const f32x16 &co, float &s1, float &s2,
                                                float &s3, float &s4)
{
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const float e = ce[v], o = co[v];
        const float e2 = e * e, o2 = o * o, w = e2 + o2;
        s1 += e;
        s2 += w;
        s3 = __builtin_fmaf(e, __builtin_fmaf(3.0f, o2, e2), s3);
        s4 = __builtin_fmaf(w, w, s4);
        s4 = __builtin_fmaf(4.0f * e2, o2, s4);
    }
}

template <int K, int PREC>
__device__ __forceinline__ void grid_power_sums_eo(const float (&x)[K], const char *lds_hi, const char *lds_lo,
                                                   int lane, float &s1, float &s2, float &s3, float &s4)
{
    constexpr int P = eo_steps<K>();
    static_assert(PREC != PREC_BF16, "weights are computed with FP32 or BF16x3 products");
    s1 = s2 = s3 = s4 = 0.0f;
    if constexpr (PREC == PREC_FP32) {
        const float4 *tab = reinterpret_cast<const float4 *>(lds_hi);
#pragma unroll 1
        for (int g = 0; g < P; ++g) {
            f32x16 ce = {}, co = {};
#pragma unroll
            for (int q = 0; q < K / 4; ++q) {
                const float4 a = tab[(g * (K / 4) + q) * kWave + lane];
                co = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, x[4 * q + 0], co, 0, 0, 0);
                ce = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, x[4 * q + 1], ce, 0, 0, 0);
                co = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, x[4 * q + 2], co, 0, 0, 0);
                ce = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, x[4 * q + 3], ce, 0, 0, 0);
            }
            pair_power_sums(ce, co, s1, s2, s3, s4);
        }
    } else {
        bf16x8 eh[P], el[P], oh[P], ol[P];
        split_eo<K, PREC>(x, eh, el, oh, ol);
        const bf16x8 *th = reinterpret_cast<const bf16x8 *>(lds_hi);
        const bf16x8 *tl = reinterpret_cast<const bf16x8 *>(lds_lo);
#pragma unroll 1
        for (int g = 0; g < P; ++g) {
            f32x16 ce = {}, co = {};
#pragma unroll
            for (int s = 0; s < P; ++s) {
                const int idx = (g * P + s) * 2 * kWave + lane;
                const bf16x8 aeh = th[idx], aoh = th[idx + kWave], ael = tl[idx], aol = tl[idx + kWave];
                ce = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ael, eh[s], ce, 0, 0, 0);
                co = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aol, oh[s], co, 0, 0, 0);
                ce = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aeh, el[s], ce, 0, 0, 0);
                co = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aoh, ol[s], co, 0, 0, 0);
                ce = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aeh, eh[s], ce, 0, 0, 0);
                co = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aoh, oh[s], co, 0, 0, 0);
            }
            pair_power_sums(ce, co, s1, s2, s3, s4);
        }
    }
    s1 *= 2.0f;
    s2 *= 2.0f;
    s3 *= 2.0f;
    s4 *= 2.0f;
}

// Per-lane sums of u~^p over this lane's grid values (p = 1..4), products in
// the requested arithmetic, from unnormalised x (the caller scales by |x|^-p).
// K >= 16 takes the half-period form.
template <int K, int PREC>
__device__ __forceinline__ void grid_power_sums(const float (&x)[K], const char *lds_hi, const char *lds_lo,
                                                int lane, float &s1, float &s2, float &s3, float &s4)
{
    if constexpr (K >= 16) {
        grid_power_sums_eo<K, PREC>(x, lds_hi, lds_lo, lane, s1, s2, s3, s4);
        return;
    }
    s1 = s2 = s3 = s4 = 0.0f;
    auto fold = [&](const f32x16 &acc) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const float u = acc[v], u2 = u * u;
            s1 += u;
            s2 += u2;
            s3 = __builtin_fmaf(u2, u, s3);
            s4 = __builtin_fmaf(u2, u2, s4);
        }
    };
    constexpr int kTileUnroll = K >= 64 ? 2 : K / 8;  // grid-tile groups unrolled
    if constexpr (PREC == PREC_FP32) {
        const float4 *tab = reinterpret_cast<const float4 *>(lds_hi);
#pragma unroll kTileUnroll
        for (int t = 0; t < K / 8; ++t) {
            f32x16 acc = {};
#pragma unroll
            for (int q = 0; q < K / 4; ++q) {
                const float4 a = tab[(t * (K / 4) + q) * kWave + lane];
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, x[4 * q + 0], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, x[4 * q + 1], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, x[4 * q + 2], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, x[4 * q + 3], acc, 0, 0, 0);
            }
            fold(acc);
        }
    } else {
        bf16x8 bh[K / 8], bl[K / 8];
        split_bf16<K, PREC>(x, bh, bl);
        const bf16x8 *th = reinterpret_cast<const bf16x8 *>(lds_hi);
        const bf16x8 *tl = reinterpret_cast<const bf16x8 *>(lds_lo);
#pragma unroll kTileUnroll
        for (int t = 0; t < K / 8; ++t) {
            f32x16 acc = {};
#pragma unroll
            for (int s = 0; s < K / 8; ++s) {
                const int idx = (t * (K / 8) + s) * kWave + lane;
                const bf16x8 ah = th[idx];
                if constexpr (PREC == PREC_BF16X3) {
                    const bf16x8 al = tl[idx];
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[s], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[s], acc, 0, 0, 0);
                }
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[s], acc, 0, 0, 0);
            }
            fold(acc);
        }
    }
}

template <int K, int PREC, int PROP>
__global__ void __launch_bounds__(kBlock) k_sir_weights(SirArgs a)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    constexpr int tab = sir_tab_bytes<K, PREC>();
    if constexpr (K >= 16) {
        stage_eo_tables<K, PREC, kBlock>(lds, a.phi_hi, a.phi_lo);
    } else {
        const uint4 *s0 = reinterpret_cast<const uint4 *>(a.phi_hi);
        uint4 *d = reinterpret_cast<uint4 *>(lds);
        for (int v = threadIdx.x; v < tab / 16; v += kBlock) d[v] = s0[v];
        if constexpr (PREC == PREC_BF16X3) {
            const uint4 *s1 = reinterpret_cast<const uint4 *>(a.phi_lo);
            for (int v = threadIdx.x; v < tab / 16; v += kBlock) d[tab / 16 + v] = s1[v];
        }
    }
    __syncthreads();
    const DevPoint &P = *a.pt;
    const int lane = threadIdx.x & 63, half = lane >> 5, pl = lane & 31;
    const unsigned long long gwave = (unsigned long long)blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6);
    const unsigned long long nwaves = (unsigned long long)gridDim.x * (kBlock / kWave);
    double w2 = 0.0, mx = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0, over = 0.0;
    for (unsigned long long tile = gwave; tile < a.n_tiles; tile += nwaves) {
        const unsigned long long local = tile * kTile + pl;
        const bool valid = local < a.n;
        const uint64_t i = P.i0 + local;
        float x[K];
        float t;
        uint32_t w_acc;
        const float inv = gen_xhat<K, PROP, false>(P, i, half, x, t, w_acc);
        float s1, s2, s3, s4;
        grid_power_sums<K, PREC>(x, lds, lds + tab, lane, s1, s2, s3, s4);
        const float i2 = inv * inv;
        s1 = (s1 + xor32(s1)) * inv;
        s2 = (s2 + xor32(s2)) * i2;
        s3 = (s3 + xor32(s3)) * (i2 * inv);
        s4 = (s4 + xor32(s4)) * (i2 * i2);
        const float la = log_a_f32<PROP>(P, t, s3);
        const float w = __builtin_amdgcn_exp2f(la * 1.4426950408889634f);
        const bool mine = valid && half == 0;
        if (mine) a.w[local] = w;
        const double wd = mine ? (double)w : 0.0;
        const double ts = sum64(wd);
        if (lane == 0) a.tile_sum[tile] = ts;
        w2 += wd * wd;
        mx = fmax(mx, wd);
        m1 += wd * (double)s1;
        m2 += wd * (double)s2;
        m3 += wd * (double)s3;
        m4 += wd * (double)s4;
        over += (mine && la > P.tau) ? 1.0 : 0.0;  // above 1 beyond the fast path's error
    }
    w2 = sum64(w2);
    mx = max64(mx);
    m1 = sum64(m1);
    m2 = sum64(m2);
    m3 = sum64(m3);
    m4 = sum64(m4);
    over = sum64(over);
    if (lane == 0) {
        double *o = a.wave_part + gwave * kSirPart;
        o[0] = w2;
        o[1] = mx;
        o[2] = m1;
        o[3] = m2;
        o[4] = m3;
        o[5] = m4;
        o[6] = over;
        o[7] = 0.0;
    }
}

// K = 128: the same outputs in the quarter-period layout (16 proposals per
// wave pass, two passes per 32-proposal tile; lane group g = l/16 holds modes
// K g/4 + 1 .. K g/4 + K/4).  log a takes the decision kernel's operations
// (the same draw, products and cube sum on the grid offset by half a step), so
// each weight is exp of the rejection step's fast-path log a; the power sums
// come from the same four syntheses (QuarterPowers), with S4 carried over to
// the grid xi_j = -pi + 2 pi j/N by the closed-form difference of the two
// grids.  One 512-thread workgroup per CU holds the 128 KB of tables.
template <int K, int PREC, int PROP>
__global__ void __launch_bounds__(Quarter<K>::BLOCK) k_sir_weights_q(SirArgs a)
{
    constexpr int B = Quarter<K>::BLOCK, CPL = K / 4, R = Quarter<K>::STEPS;
    constexpr int one = (PREC == PREC_FP32 ? Quarter<K>::F32_BYTES : Quarter<K>::BF16_BYTES) / 16;
    static_assert(PREC != PREC_BF16, "weights are computed with FP32 or BF16x3 products");
    extern __shared__ __attribute__((aligned(16))) char lds[];
    {
        const uint4 *s0 = reinterpret_cast<const uint4 *>(a.phi_hi);
        const uint4 *s1 = reinterpret_cast<const uint4 *>(a.phi_lo);
        uint4 *d = reinterpret_cast<uint4 *>(lds);
        for (int v = threadIdx.x; v < one; v += B) d[v] = s0[v];
        if constexpr (PREC == PREC_BF16X3)
            for (int v = threadIdx.x; v < one; v += B) d[one + v] = s1[v];
    }
    __syncthreads();
    const char *lds_hi = lds, *lds_lo = lds + (PREC == PREC_BF16X3 ? one * 16 : 0);
    const DevPoint &P = *a.pt;
    const int lane = threadIdx.x & 63, g = lane >> 4, pl = lane & 15;
    const unsigned long long gwave = (unsigned long long)blockIdx.x * (B / kWave) + (threadIdx.x >> 6);
    const unsigned long long nwaves = (unsigned long long)gridDim.x * (B / kWave);
    double w2 = 0.0, mx = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0, over = 0.0;
    for (unsigned long long tile = gwave; tile < a.n_tiles; tile += nwaves) {
        double ts = 0.0;
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            const unsigned long long local = tile * kTile + 16 * h + pl;
            const bool valid = local < a.n;
            const uint64_t i = P.i0 + local;
            const uint32_t c0 = (uint32_t)i, c1 = (uint32_t)(i >> 32);
            float r2 = 0.0f, a1 = 0.0f, a2 = 0.0f, top_c, top_s;
            QuarterPowers pw;
            auto fold = [&](const f32x4 &ce, const f32x4 &co, const f32x4 &se, const f32x4 &so) {
                pw.fold(ce, co, se, so);
            };
            if constexpr (PREC == PREC_FP32) {
                float c[CPL], s[CPL];
                gen_block128<K, PROP>(P, c0, c1, g, 0, c, r2, a1, a2);
                gen_block128<K, PROP>(P, c0, c1, g, 1, s, r2, a1, a2);
                top_c = c[CPL - 1];
                top_s = s[CPL - 1];
                quarter_tiles_f32<K>(c, s, lds_hi, lane, fold);
            } else {
                bf16x8 bh[4][R], bl[4][R];
#pragma unroll
                for (int blk = 0; blk < 2; ++blk) {
                    float v[CPL];
                    gen_block128<K, PROP>(P, c0, c1, g, blk, v, r2, a1, a2);
                    if (blk == 0) top_c = v[CPL - 1];
                    else top_s = v[CPL - 1];
#pragma unroll
                    for (int odd = 0; odd < 2; ++odd)
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            quarter_operand<CPL, true>(v, odd, r, bh[2 * blk + odd][r], bl[2 * blk + odd][r]);
                    __builtin_amdgcn_sched_barrier(0);
                }
                quarter_tiles_bf16<K, PREC>(bh, bl, lds_hi, lds_lo, lane, fold);
            }
            float s1, s2, s3, s4;
            pw.result(s1, s2, s3, s4);
            if (g == 3) s4 += s4_grid_correction<K>(top_c, top_s);  // mode K: last coordinate of group 3
            float t;
            const float inv = finish_norm128<K>(g, r2, a1, a2, t);
            const float i2 = inv * inv;
            s1 = sum4(s1) * inv;
            s2 = sum4(s2) * i2;
            s3 = sum4(s3) * (inv * inv * inv);  // as the decision kernel
            s4 = sum4(s4) * (i2 * i2);
            const float la = log_a_f32<PROP>(P, t, s3);
            const float w = __builtin_amdgcn_exp2f(la * 1.4426950408889634f);
            const bool mine = valid && g == 0;
            if (mine) a.w[local] = w;
            const double wd = mine ? (double)w : 0.0;
            ts += sum64(wd);
            w2 += wd * wd;
            mx = fmax(mx, wd);
            m1 += wd * (double)s1;
            m2 += wd * (double)s2;
            m3 += wd * (double)s3;
            m4 += wd * (double)s4;
            over += (mine && la > P.tau) ? 1.0 : 0.0;  // above 1 beyond the fast path's error
        }
        if (lane == 0) a.tile_sum[tile] = ts;
    }
    w2 = sum64(w2);
    mx = max64(mx);
    m1 = sum64(m1);
    m2 = sum64(m2);
    m3 = sum64(m3);
    m4 = sum64(m4);
    over = sum64(over);
    if (lane == 0) {
        double *o = a.wave_part + gwave * kSirPart;
        o[0] = w2;
        o[1] = mx;
        o[2] = m1;
        o[3] = m2;
        o[4] = m3;
        o[5] = m4;
        o[6] = over;
        o[7] = 0.0;
    }
}

// The cumulative sums must be monotone in the proposal index, so that the
// draw ranges of consecutive tiles never overlap: every level adds
// non-negative terms sequentially (FP rounding is monotone), and a fixed FP64
// offset is added to each of a sequence of increasing values.

// Exclusive prefix of 256 FP64 values in LDS, summed sequentially by thread
// 0; returns the total.
__device__ double block_exclusive_seq(double *s, int tid)
{
    __shared__ double total;
    __syncthreads();
    if (tid == 0) {
        double run = 0.0;
        for (int k = 0; k < 256; ++k) {
            const double v = s[k];
            s[k] = run;
            run += v;
        }
        total = run;
    }
    __syncthreads();
    return total;
}

// Level 1: block b covers tiles [b kSirChunk, (b + 1) kSirChunk); thread t
// takes 16 consecutive tiles in order.
__global__ void __launch_bounds__(256) k_sir_scan_chunks(SirArgs a)
{
    __shared__ double s[256];
    const int tid = threadIdx.x;
    const unsigned long long t0 = (unsigned long long)blockIdx.x * kSirChunk + (unsigned long long)tid * 16;
    double loc[16];
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const unsigned long long t = t0 + q;
        const double v = t < a.n_tiles ? a.tile_sum[t] : 0.0;
        loc[q] = acc;  // exclusive within the thread
        acc += v;
    }
    s[tid] = acc;
    const double total = block_exclusive_seq(s, tid);
    const double before = s[tid];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const unsigned long long t = t0 + q;
        if (t < a.n_tiles) a.tile_off[t] = before + loc[q];
    }
    if (tid == 0) a.chunk_sum[blockIdx.x] = total;
}

// Level 2: the chunk sums in one sequential pass (one FP64 add per kSirChunk
// tiles); chunk_off[n_chunks] is the grand total.
__global__ void __launch_bounds__(64) k_sir_scan_top(SirArgs a)
{
    if (threadIdx.x != 0) return;
    double run = 0.0;
    for (unsigned long long c = 0; c < a.n_chunks; ++c) {
        a.chunk_off[c] = run;
        run += a.chunk_sum[c];
    }
    a.chunk_off[a.n_chunks] = run;
}

__global__ void __launch_bounds__(256) k_sir_scan_add(SirArgs a)
{
    for (unsigned long long t = (unsigned long long)blockIdx.x * 256 + threadIdx.x; t < a.n_tiles;
         t += (unsigned long long)gridDim.x * 256)
        a.tile_off[t] += a.chunk_off[t / kSirChunk];
}

__device__ __forceinline__ unsigned long long draw_of(double c, const SirArgs &a, unsigned long long lo,
                                                      unsigned long long hi)
{
    const double v = ceil(c * a.scale - a.u0);
    unsigned long long r = v <= 0.0 ? 0ull : (v >= (double)a.m ? a.m : (unsigned long long)v);
    return r < lo ? lo : (r > hi ? hi : r);
}

// QROWS (K = 128): the rows of x^ from the quarter-period draw (gen_x128, the
// sampler's rows), proposal 16 h + l % 16 of the tile in lanes l, h = 0, 1.
template <int K, int PROP, bool QROWS>
__global__ void __launch_bounds__(kBlock) k_sir_resample(SirArgs a)
{
    const DevPoint &P = *a.pt;
    const int lane = threadIdx.x & 63, half = lane >> 5, pl = lane & 31;
    const unsigned long long gwave = (unsigned long long)blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6);
    const unsigned long long nwaves = (unsigned long long)gridDim.x * (kBlock / kWave);
    for (unsigned long long tile = gwave; tile < a.n_tiles; tile += nwaves) {
        const double off = a.tile_off[tile];
        const bool last_tile = tile + 1 == a.n_tiles;
        const unsigned long long A0 = draw_of(off, a, 0ull, a.m);
        const unsigned long long A1 = last_tile ? a.m : draw_of(a.tile_off[tile + 1], a, 0ull, a.m);
        if (__builtin_amdgcn_readfirstlane((int)(A1 <= A0))) continue;  // no draw in this tile
        const unsigned long long local = tile * kTile + pl;
        const bool valid = local < a.n;
        const double w = (half == 0 && valid) ? (double)a.w[local] : 0.0;
        // prefix over the tile's 32 proposals, summed sequentially (monotone)
        double run = 0.0, excl = 0.0, incl = 0.0;
#pragma unroll
        for (int q = 0; q < kTile; ++q) {
            const double v = __shfl(w, q, 64);
            if (pl == q) excl = run;
            run += v;
            if (pl == q) incl = run;
        }
        const unsigned long long n_in = a.n - tile * kTile;  // valid proposals of the tile (>= 1)
        const int last = (int)(n_in < (unsigned long long)kTile ? n_in - 1 : kTile - 1);
        unsigned long long r0 = pl == 0 ? A0 : draw_of(off + excl, a, A0, A1);
        unsigned long long r1 = pl == last ? A1 : draw_of(off + incl, a, A0, A1);
        if (half != 0 || !valid || r1 < r0) r1 = r0;
        // the sin-block lanes take the draws of their proposal
        const unsigned long long q0 = __shfl(r0, pl, 64), q1 = __shfl(r1, pl, 64);
        const uint64_t i = P.i0 + local;
        if (half == 0)
            for (unsigned long long r = q0; r < q1; ++r) a.index[r] = i;
        if (a.xhat && __ballot(q1 > q0) != 0ull) {
            if constexpr (QROWS) {
                constexpr int CPL = K / 4;
                const int g = lane >> 4;
#pragma unroll 1
                for (int h = 0; h < 2; ++h) {
                    const int pp = 16 * h + (lane & 15);  // proposal of the tile
                    const unsigned long long d0 = __shfl(r0, pp, 64), d1 = __shfl(r1, pp, 64);
                    if (__ballot(d1 > d0) == 0ull) continue;
                    float c[CPL], s[CPL], t;
                    uint32_t w_acc;
                    gen_x128<K, PROP, true>(P, P.i0 + tile * kTile + pp, g, c, s, t, w_acc);
                    for (unsigned long long r = d0; r < d1; ++r) {
                        float *dst = a.xhat + r * (2 * K) + CPL * g;
#pragma unroll
                        for (int j = 0; j < CPL; ++j) {
                            dst[j] = c[j];
                            dst[K + j] = s[j];
                        }
                    }
                }
            } else {
                float x[K];
                float t;
                uint32_t w_acc;
                gen_xhat<K, PROP, true>(P, i, half, x, t, w_acc);
                for (unsigned long long r = q0; r < q1; ++r) {
                    float *dst = a.xhat + r * (2 * K) + half * K;
#pragma unroll
                    for (int j = 0; j < K; ++j) dst[j] = x[j];
                }
            }
        }
    }
}

}  // namespace

int sir_block(int K) { return K == 128 ? Quarter<128>::BLOCK : kBlock; }
int sir_waves(int K, int n_cu)
{
    return K == 128 ? n_cu * (Quarter<128>::BLOCK / kWave) : 4 * n_cu * (kBlock / kWave);
}

template <int PREC, int PROP>
hipError_t launch_sir_weights_q128(const SirArgs &a, int n_cu, hipStream_t st)
{
    constexpr int K = 128;
    constexpr int lds = PREC == PREC_FP32 ? Quarter<K>::F32_BYTES : 2 * Quarter<K>::BF16_BYTES;
    auto kern = k_sir_weights_q<K, PREC, PROP>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    // one workgroup per CU (the tables fill LDS): sir_waves(128, n_cu) waves
    hipLaunchKernelGGL(kern, dim3(n_cu), dim3(Quarter<K>::BLOCK), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_sir_weights(int K, int prec, int proposal, const SirArgs &a, int n_cu, hipStream_t st)
{
    if (K == 128) {
        if (prec == PREC_FP32)
            return proposal == PROP_SIGMA ? launch_sir_weights_q128<PREC_FP32, PROP_SIGMA>(a, n_cu, st)
                                          : launch_sir_weights_q128<PREC_FP32, PROP_UNIFORM>(a, n_cu, st);
        if (prec == PREC_BF16X3)
            return proposal == PROP_SIGMA ? launch_sir_weights_q128<PREC_BF16X3, PROP_SIGMA>(a, n_cu, st)
                                          : launch_sir_weights_q128<PREC_BF16X3, PROP_UNIFORM>(a, n_cu, st);
        return hipErrorInvalidValue;
    }
    const int grid = 4 * n_cu;  // sir_waves(K, n_cu) waves
#define TKDV_SIRW(KK, PR, PP)                                                                            \
    if (K == KK && prec == PR && proposal == PP) {                                                       \
        constexpr int tab = sir_tab_bytes<KK, PR>();                                                     \
        constexpr int lds = PR == PREC_BF16X3 ? 2 * tab : tab;                                           \
        auto kern = k_sir_weights<KK, PR, PP>;                                                           \
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds); \
        if (e != hipSuccess) return e;                                                                   \
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, st, a);                                  \
        return hipGetLastError();                                                                        \
    }
#define TKDV_SIRW_K(KK)                                                                                  \
    TKDV_SIRW(KK, PREC_FP32, PROP_UNIFORM) TKDV_SIRW(KK, PREC_FP32, PROP_SIGMA)                          \
    TKDV_SIRW(KK, PREC_BF16X3, PROP_UNIFORM) TKDV_SIRW(KK, PREC_BF16X3, PROP_SIGMA)
    TKDV_SIRW_K(8) TKDV_SIRW_K(16) TKDV_SIRW_K(32) TKDV_SIRW_K(64)
#undef TKDV_SIRW_K
#undef TKDV_SIRW
    return hipErrorInvalidValue;
}

hipError_t launch_sir_scan(const SirArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_sir_scan_chunks, dim3((unsigned)a.n_chunks), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sir_scan_top, dim3(1), dim3(64), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned long long g = (a.n_tiles + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_sir_scan_add, dim3((unsigned)g), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_sir_resample(int K, int proposal, const SirArgs &a, int n_cu, hipStream_t st)
{
    const dim3 g(12 * n_cu), b(kBlock);  // three waves per SIMD: the tile scan is latency-bound
#define TKDV_SIRR(KK)                                                                                    \
    if (K == KK) {                                                                                       \
        if (proposal == PROP_SIGMA) hipLaunchKernelGGL((k_sir_resample<KK, PROP_SIGMA, KK == 128>), g, b, 0, st, a); \
        else hipLaunchKernelGGL((k_sir_resample<KK, PROP_UNIFORM, KK == 128>), g, b, 0, st, a);                    \
        return hipGetLastError();                                                                        \
    }
    TKDV_SIRR(8) TKDV_SIRR(16) TKDV_SIRR(32) TKDV_SIRR(64) TKDV_SIRR(128)
#undef TKDV_SIRR
    return hipErrorInvalidValue;
}

}  // namespace tkdv
