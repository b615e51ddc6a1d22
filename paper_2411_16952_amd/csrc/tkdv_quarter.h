// Quarter-period form of the synthesis at K = 64 and 128 (N = 256, 512):
// device helpers shared by the decision, output, SIR and synthesis kernels.
//
// Layout.  One wavefront evaluates a tile of 16 proposals; proposal p of the
// tile lives in lanes p + 16 g, g = 0..3, and lane group g holds the cos and
// sin coordinates of the K/4 modes K g/4 + 1 .. K g/4 + K/4 (c[j] =
// x_{Kg/4+j+1}, s[j] = x_{K+Kg/4+j+1}).  That is the operand layout of the 16x16x32 BF16
// (and 16x16x4 FP32) matrix instructions with the proposals as the B
// (column) operand: lane l supplies k-rows 8 (l/16) .. 8 (l/16) + 7 of column
// l % 16, and receives rows 4 (l/16) .. 4 (l/16) + 3 of the result.
//
// Quarter-period synthesis.  H3 = (1/6) int u^3 dxi (Sec. II.A) is the
// trapezoid sum of u^3 on any equispaced grid of N >= 3K + 1 points; the
// decision kernels take the grid offset by half a step, xi_j = -pi + 2 pi (j + 1/2)/N,
// whose points come in orbits {xi, -xi, xi + pi, pi - xi} with one
// representative in (0, pi/2): xi_rho = pi (2 rho + 1)/N, rho < N/4.  With Ce,
// Co (cos block, even / odd modes) and Se, So (sin block) at a representative,
// the four field values are (Ce + Co) +- (Se + So) and (Ce - Co) +- (Se - So),
// and their cubes sum to 4 Ce (Ce^2 + 3 Co^2 + 3 Se^2 + 3 So^2) + 24 Co Se So.
// The tables carry the Co, Se, So rows times sqrt(3) (co = sqrt 3 Co, ...):
// 4 Ce (Ce^2 + co^2 + se^2 + so^2) + (8/sqrt 3) co se so.  Each of the four
// syntheses contracts K/2 coordinates: a quarter of the plain product's matrix
// work, and tables of N/4 x 2K entries (64 KB per BF16 table at K = 128) that
// fit in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include "tkdv_device.h"
#include "tkdv_internal.h"

namespace tkdv {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int kTile16 = 16;            // proposals per wave tile

// Sizes of the quarter-period form at K (64 or 128): CPL coordinates of each
// block per lane, K/16 tiles of 16 representatives (N/4 = K of them), K/64
// BF16 k-steps and K/32 groups of four FP32 k-steps per synthesis.
template <int K>
struct Quarter {
    static constexpr int CPL = K / 4;
    static constexpr int NB = CPL / 4;        // Philox blocks of one block's coordinates per lane
    static constexpr int TILES = K / 16;
    static constexpr int STEPS = K / 64;      // BF16 k-steps (32 k-rows, 8 per lane group)
    static constexpr int QG = K / 32;         // FP32 k-steps in groups of 4
    // bytes of one table: BF16 [tile][out][step][64 lanes][8], FP32 [tile][out][group][64 lanes][4]
    static constexpr int BF16_BYTES = TILES * 4 * STEPS * 64 * 16;
    static constexpr int F32_BYTES = TILES * 4 * QG * 64 * 16;
    // workgroup of the kernels that hold a whole proposal's power sums (the
    // SIR weights, the synthesis, the verification instantiation of the
    // decision kernel): at K = 128 the 128 KB of tables leave one workgroup
    // per CU, 8 waves (2 per SIMD) with every register they need; at K = 64
    // (32 KB) workgroups of 256.  The sampling decision kernel takes
    // decide_block(K).
    static constexpr int BLOCK = K == 128 ? 512 : 256;
    static constexpr int lds(int prec) { return prec == PREC_FP32 ? F32_BYTES : 2 * BF16_BYTES; }
};

__device__ __forceinline__ unsigned long long wave_sum_u64_128(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_max_128(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_sum_f64_128(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ unsigned long long bcast0(unsigned long long v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}
// sum over the four lanes of a proposal (l, l^16, l^32, l^48); every lane
// gets the same two operands in the last addition, hence the same bits
__device__ __forceinline__ float sum4(float v)
{
    v = v + __shfl_xor(v, 16, 64);
    return v + __shfl_xor(v, 32, 64);
}


// Block b (0: cos, 1: sin) of proposal i for this lane: the K/4 coordinates
// of modes K g/4 + 1 .. K g/4 + K/4 (coordinate m from word m, Box-Muller on
// word pairs; X = Sigma^{1/2} z for the paper's proposal), and their
// contributions to |X|^2, sum (j+1) X^2 and sum (j+1)^2 X^2 (t = sum k^2 X_k^2
// over both blocks, k = K g/4 + j + 1).  FAST: the Box-Muller form of the
// decision and weight kernels (box_muller_f32).
template <int K, int PROP, bool FAST = true>
__device__ __forceinline__ void gen_block128(const DevPoint &P, uint32_t c0, uint32_t c1, int g, int b,
                                             float (&v)[K / 4], float &r2, float &a1, float &a2)
{
    constexpr int NB = Quarter<K>::NB;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const uint4 w = philox4x32_10(c0, c1, P.point_id, (uint32_t)(b * (K / 4) + NB * g + q), P.key0, P.key1);
        box_muller_f32<FAST>(w.x, w.y, v[4 * q + 0], v[4 * q + 1]);
        box_muller_f32<FAST>(w.z, w.w, v[4 * q + 2], v[4 * q + 3]);
    }
    if (PROP == PROP_SIGMA) {
        const float4 *sg = reinterpret_cast<const float4 *>(P.sig + (K / 4) * g);
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const float4 sv = sg[q];
            v[4 * q + 0] *= sv.x;
            v[4 * q + 1] *= sv.y;
            v[4 * q + 2] *= sv.z;
            v[4 * q + 3] *= sv.w;
        }
    }
#pragma unroll
    for (int j = 0; j < K / 4; ++j) {
        const float q = v[j] * v[j];
        r2 += q;
        a1 = __builtin_fmaf((float)(j + 1), q, a1);
        a2 = __builtin_fmaf((float)((j + 1) * (j + 1)), q, a2);
    }
}

// |X|^-1 and t of the projected point from the lane's partial sums (the four
// lanes of a proposal end with bitwise identical values).
template <int K>
__device__ __forceinline__ float finish_norm128(int g, float r2, float a1, float a2, float &t)
{
    const float b = (float)((K / 4) * g);
    float tk = __builtin_fmaf(b * b, r2, __builtin_fmaf(2.0f * b, a1, a2));
    r2 = sum4(r2);
    tk = sum4(tk);
    const float inv = __builtin_amdgcn_rsqf(r2);
    t = tk * (inv * inv);
    return inv;
}

// Proposal i of the point: this lane's K/4 cos and K/4 sin coordinates of X
// (words 0..2K-1 as in every sampler: coordinate m from word m, Box-Muller on
// word pairs; X = Sigma^{1/2} z for the paper's proposal), |X|^-1, t of the
// projected point and the acceptance word (word 2K).  With NORMALIZE the
// coordinates are projected onto the sphere (rows for the caller, drawn with
// the folded-word Box-Muller form unless FAST).  The four lanes of a proposal
// hold bitwise identical |X|^2 and t.
template <int K, int PROP, bool NORMALIZE, bool FAST = !NORMALIZE>
__device__ __forceinline__ float gen_x128(const DevPoint &P, uint64_t i, int g, float (&c)[K / 4],
                                          float (&s)[K / 4], float &t, uint32_t &w_acc)
{
    const uint32_t c0 = (uint32_t)i, c1 = (uint32_t)(i >> 32);
    float r2 = 0.0f, a1 = 0.0f, a2 = 0.0f;
    gen_block128<K, PROP, FAST>(P, c0, c1, g, 0, c, r2, a1, a2);
    gen_block128<K, PROP, FAST>(P, c0, c1, g, 1, s, r2, a1, a2);
    w_acc = philox4x32_10(c0, c1, P.point_id, (uint32_t)(K / 2), P.key0, P.key1).x;
    const float inv = finish_norm128<K>(g, r2, a1, a2, t);
    if (NORMALIZE) {
#pragma unroll
        for (int j = 0; j < K / 4; ++j) {
            c[j] *= inv;
            s[j] *= inv;
        }
    }
    return inv;
}

// The cube sums of one representative from its four syntheses (co, se, so
// carry sqrt(3)): s1 += Ce (Ce^2 + co^2 + se^2 + so^2), s2 += co se so.
__device__ __forceinline__ void quarter_cubes(const f32x4 &ce, const f32x4 &co, const f32x4 &se, const f32x4 &so,
                                              float &s1, float &s2)
{
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const float e = ce[v];
        const float q = __builtin_fmaf(co[v], co[v], __builtin_fmaf(se[v], se[v], __builtin_fmaf(so[v], so[v], e * e)));
        s1 = __builtin_fmaf(e, q, s1);
        s2 = __builtin_fmaf(co[v] * se[v], so[v], s2);
    }
}

// BF16 operands of one contraction (out o: 0 Ce, 1 Co, 2 Se, 3 So), k-step r:
// entry e = the coordinate of mode K g/4 + 2 (8 r + e) + 2 (even) or + 1 (odd).
template <int N, bool LO>
__device__ __forceinline__ void quarter_operand(const float (&v)[N], int odd, int r, bf16x8 &hi, bf16x8 &lo)
{
    u32x4_t wh, wl = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const int j0 = 16 * r + 4 * w + (odd ? 0 : 1);  // entries 2w, 2w + 1: coordinates j0, j0 + 2
        wh[w] = pack_hi(v[j0], v[j0 + 2]);
        if (LO) wl[w] = pack_lo(v[j0], v[j0 + 2], wh[w]);
    }
    hi = __builtin_bit_cast(bf16x8, wh);
    lo = __builtin_bit_cast(bf16x8, wl);
}

// The four syntheses Ce, co, se, so (FP32 products) of each tile of 16
// representatives of the offset grid, from unprojected coordinates; fold gets
// the tile's accumulators (element v of lane l: representative 16 tau +
// 4 (l/16) + v, proposal l % 16).  k-step sg of out o reads coordinate 2 sg + 1
// (even mode) or 2 sg (odd mode) of the block.
template <int K, class Fold>
__device__ __forceinline__ void quarter_tiles_f32(const float (&c)[K / 4], const float (&s)[K / 4],
                                                  const char *lds_hi, int lane, Fold &&fold)
{
    constexpr int QG = Quarter<K>::QG;
    const float4 *tab = reinterpret_cast<const float4 *>(lds_hi);
#pragma unroll 1
    for (int tau = 0; tau < Quarter<K>::TILES; ++tau) {
        f32x4 acc[4] = {f32x4{}, f32x4{}, f32x4{}, f32x4{}};
#pragma unroll
        for (int q4 = 0; q4 < QG; ++q4)
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                const float4 a = tab[((tau * 4 + o) * QG + q4) * 64 + lane];
                const float *v = (o < 2) ? c : s;
                const int par = (o == 0 || o == 2) ? 1 : 0;
                acc[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, v[2 * (4 * q4 + 0) + par], acc[o], 0, 0, 0);
                acc[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, v[2 * (4 * q4 + 1) + par], acc[o], 0, 0, 0);
                acc[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, v[2 * (4 * q4 + 2) + par], acc[o], 0, 0, 0);
                acc[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, v[2 * (4 * q4 + 3) + par], acc[o], 0, 0, 0);
            }
        fold(acc[0], acc[1], acc[2], acc[3]);
    }
}

// The same from BF16 operands [out][step] (hi, and lo for BF16x3) with FP32
// accumulation; UNR tiles per loop trip (two let one tile's products run
// beside the previous tile's fold).
template <int K, int PREC, class Fold, int UNR = 1>
__device__ __forceinline__ void quarter_tiles_bf16(const bf16x8 (&bh)[4][K / 64], const bf16x8 (&bl)[4][K / 64],
                                                   const char *lds_hi, const char *lds_lo, int lane, Fold &&fold)
{
    constexpr int R = Quarter<K>::STEPS;
    constexpr int TILE = 4 * R * 64;  // entries of one tile's table
#pragma unroll UNR
    for (int tau = 0; tau < Quarter<K>::TILES; ++tau) {
        // this tile's entry offset, opaque to the compiler: the two tables'
        // reads then address from one base each with immediate offsets, not a
        // separate addition for every read past 64 KB (K = 128)
        uint32_t e = (uint32_t)(tau * TILE + lane) * (uint32_t)sizeof(bf16x8);  // bytes
        asm volatile("" : "+v"(e));
        const bf16x8 *th = reinterpret_cast<const bf16x8 *>(lds_hi + e);
        const bf16x8 *tl = reinterpret_cast<const bf16x8 *>(lds_lo + e);
        f32x4 acc[4] = {f32x4{}, f32x4{}, f32x4{}, f32x4{}};
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                const int idx = (o * R + r) * 64;
                const bf16x8 ah = th[idx];
                if constexpr (PREC == PREC_BF16X3) {
                    const bf16x8 al = tl[idx];
                    acc[o] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[o][r], acc[o], 0, 0, 0);
                    acc[o] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[o][r], acc[o], 0, 0, 0);
                }
                acc[o] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[o][r], acc[o], 0, 0, 0);
            }
        fold(acc[0], acc[1], acc[2], acc[3]);
    }
}

// S3 = sum over the N = 4K offset-grid values of u~^3 for this lane's share
// (the caller sums the four lanes), from unprojected coordinates, FP32 products.
template <int K>
__device__ __forceinline__ float cube_sum_q128_f32(const float (&c)[K / 4], const float (&s)[K / 4],
                                                   const char *lds_hi, int lane)
{
    float s1 = 0.0f, s2 = 0.0f;
    quarter_tiles_f32<K>(c, s, lds_hi, lane,
                         [&](const f32x4 &ce, const f32x4 &co, const f32x4 &se, const f32x4 &so) {
                             quarter_cubes(ce, co, se, so, s1, s2);
                         });
    return __builtin_fmaf(4.0f, s1, 4.6188021535170061f * s2);  // 4 s1 + (8/sqrt 3) s2
}

// The same from BF16 operands.
template <int K, int PREC, int UNR = 1>
__device__ __forceinline__ float cube_sum_q128_bf16(const bf16x8 (&bh)[4][K / 64], const bf16x8 (&bl)[4][K / 64],
                                                    const char *lds_hi, const char *lds_lo, int lane)
{
    float s1 = 0.0f, s2 = 0.0f;
    auto fold = [&](const f32x4 &ce, const f32x4 &co, const f32x4 &se, const f32x4 &so) {
        quarter_cubes(ce, co, se, so, s1, s2);
    };
    quarter_tiles_bf16<K, PREC, decltype(fold) &, UNR>(bh, bl, lds_hi, lds_lo, lane, fold);
    return __builtin_fmaf(4.0f, s1, 4.6188021535170061f * s2);  // 4 s1 + (8/sqrt 3) s2
}

// Power sums S_p = sum of u~^p over the four points of every orbit, p = 1..4,
// from the four syntheses (co, se, so carry sqrt 3).  With Co = co/sqrt 3, ...
// and u~ = Ce + a Co + b Se + a b So over a, b = +-1:
//   sum u~   = 4 Ce,
//   sum u~^2 = 4 (Ce^2 + Co^2 + Se^2 + So^2) = (4/3) (2 Ce^2 + Q),
//   sum u~^3 = 4 Ce Q + (8/sqrt 3) co se so                        (quarter_cubes),
//   sum u~^4 = 4 (Ce^4 + Co^4 + Se^4 + So^4) + 24 (the six products of two
//              squares) + 96 Ce Co Se So
//            = 4 (Q^2 - (8/9) sg^2 + (4/9) m) + (32/sqrt 3) Ce co se so,
// where Q = Ce^2 + co^2 + se^2 + so^2, sg = co^2 + se^2 + so^2 and m =
// co^2 se^2 + co^2 so^2 + se^2 so^2.  The cube sums take the operations of
// quarter_cubes unchanged.
struct QuarterPowers {
    float e1 = 0.0f, e2 = 0.0f, c1 = 0.0f, c2 = 0.0f, f4 = 0.0f, f4x = 0.0f;
    __device__ __forceinline__ void fold(const f32x4 &ce, const f32x4 &co, const f32x4 &se, const f32x4 &so)
    {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float e = ce[v];
            const float q = __builtin_fmaf(co[v], co[v], __builtin_fmaf(se[v], se[v], __builtin_fmaf(so[v], so[v], e * e)));
            const float cse = co[v] * se[v];
            c1 = __builtin_fmaf(e, q, c1);
            c2 = __builtin_fmaf(cse, so[v], c2);
            e1 += e;
            e2 += __builtin_fmaf(2.0f * e, e, q);
            const float p2 = co[v] * co[v], q2 = se[v] * se[v], r2 = so[v] * so[v];
            const float sg = p2 + q2 + r2;
            const float m = __builtin_fmaf(p2, q2, __builtin_fmaf(p2, r2, q2 * r2));
            f4 = __builtin_fmaf(q, q, f4);
            f4 = __builtin_fmaf(-0.88888888888888889f * sg, sg, f4);
            f4 = __builtin_fmaf(0.44444444444444444f, m, f4);
            f4x = __builtin_fmaf(e * cse, so[v], f4x);
        }
    }
    // this lane's shares of S1..S4
    __device__ __forceinline__ void result(float &s1, float &s2, float &s3, float &s4) const
    {
        s1 = 4.0f * e1;
        s2 = 1.3333333333333333f * e2;
        s3 = __builtin_fmaf(4.0f, c1, 4.6188021535170061f * c2);  // as cube_sum_q128_*
        s4 = __builtin_fmaf(4.0f, f4, 18.475208614068024f * f4x);
    }
};

// The sums over the grid xi_j = -pi + 2 pi j/N instead: p <= 3 are the same
// (u~^p has no frequency N, both trapezoid sums are exact); u~^4 reaches
// frequency N = 4K through the top mode alone, and the two grids differ by
// (N/4) Re((a_K - i b_K)^4) = (N/4) (a^4 - 6 a^2 b^2 + b^4) (a = x_K, b = x_2K,
// unprojected): added by the lane group holding mode K.
template <int K>
__device__ __forceinline__ float s4_grid_correction(float a, float b)
{
    const float a2 = a * a, b2 = b * b;
    return (float)K * __builtin_fmaf(a2, a2, __builtin_fmaf(-6.0f * a2, b2, b2 * b2));
}

}  // namespace tkdv
