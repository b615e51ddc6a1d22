// Device building blocks of the gfx950 TKdV rejection sampler.
//
// One wavefront evaluates a tile of 32 proposals; proposal p of the tile lives
// in lanes p (cos block: coordinates x^_1..x^_K) and p + 32 (sin block:
// x^_{K+1}..x^_{2K}).  This is exactly the operand layout of the 32x32 matrix
// instructions with the proposals as the B (column) operand, so the
// spectral-to-grid synthesis u~ = Phi^T x^ needs no data movement, and each
// lane ends up holding half of its proposal's grid values.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tkdv_internal.h"

namespace tkdv {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

enum { PREC_FP32 = 0, PREC_BF16 = 1, PREC_BF16X3 = 2 };
enum { PROP_UNIFORM = 0, PROP_SIGMA = 1, PROP_MIXTURE = 2 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): per round two 32x32->64 products of
// counter words 0 and 2 with the two multipliers, high halves XORed with the
// other counter words and the key, key advanced by the Weyl constants.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 multiply instruction per product
        const uint64_t pa = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t pb = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t hi_a = (uint32_t)(pa >> 32), lo_a = (uint32_t)pa;
        const uint32_t hi_b = (uint32_t)(pb >> 32), lo_b = (uint32_t)pb;
        uint32_t n0 = __builtin_amdgcn_bitop3_b32(hi_b, c1, k0, 0x96);  // three-way xor
        uint32_t n2 = __builtin_amdgcn_bitop3_b32(hi_a, c3, k1, 0x96);
        c0 = n0; c1 = lo_b; c2 = n2; c3 = lo_a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// ---------------------------------------------------------------------------
// FP32 transforms of the 32-bit words.  U = (w + 1/2) 2^-32.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float log2_hw(float x) { return __builtin_amdgcn_logf(x); }

// -2 ln U of a word, U = (w + 1/2) 2^-32, with one hardware log2:
//   U < 1/2:  log2(U) (relative accuracy of the hardware log2, |ln U| > ln 2);
//   U >= 1/2: d = 1 - U is formed exactly from ~w; for d < 2^-12 the series
//             -2 ln(1 - d) = 2d + d^2 (+ 2d^3/3 + ...: truncation below d^2/3
//             <= 2^-24/3 relative), otherwise log2(1 - d) with 1 - d rounded.
//             There the absolute error of -2 ln U is ~1e-7, and with
//             r = sqrt(-2 ln U) >= 0.022 the error of r stays below 1.4e-6.
__device__ __forceinline__ float neg2_log_u_word(uint32_t w)
{
    const float two_m32 = 2.3283064365386963e-10f;
    const bool upper = (w & 0x80000000u) != 0u;
    // q = U for U < 1/2 and q = d = 1 - U for U >= 1/2 (~w = 2^32 - 1 - w), one conversion
    const uint32_t v = w ^ (uint32_t)((int32_t)w >> 31);
    const float q = __builtin_fmaf((float)v, two_m32, 0.5f * two_m32);
    const float d = q, u = q;
    const float ser = __builtin_fmaf(d, d, d + d);
    const float lg = log2_hw(upper ? 1.0f - d : u) * -1.3862943611198906f;  // -2 ln 2
    return (upper && d < 0x1p-12f) ? ser : lg;
}

// -log2 U = (-2 ln U)/(2 ln 2) of a word, five instructions fewer than
// neg2_log_u_word with its error bound (the last bits differ): the word read
// as a signed integer s (s = w - 2^32 for w >= 2^31) gives qs = (s + 1/2) 2^-32,
// which is U below 1/2 and -(1 - U) above, both exact while |s| < 2^24, so one
// conversion yields d = |qs| without the integer fold; fract(qs) is the log's
// argument (U, or 1 - d rounded) without a subtraction and a selection; and
// the factor 2 ln 2 is left out.  Series below d = 2^-12, i.e. for words
// w >= 2^32 - 2^20 (one integer comparison):
// -log2(1 - d) = d (1 + d/2)/ln 2, truncation below d^2/3 relative.
__device__ __forceinline__ float neg_log2_u_word_signed(uint32_t w)
{
    const float two_m32 = 2.3283064365386963e-10f;
    const float qs = __builtin_fmaf((float)(int32_t)w, two_m32, 0.5f * two_m32);
    const float d = __builtin_fabsf(qs);
    const float ser = d * __builtin_fmaf(d, 0.72134752044448170f, 1.4426950408889634f);  // 1/(2 ln 2), 1/ln 2
    const float lg = -log2_hw(__builtin_amdgcn_fractf(qs));
    return w >= 0xFFF00000u ? ser : lg;
}

// ln U of a word (the same arithmetic, scaled by -1/2).
__device__ __forceinline__ float log_u_word(uint32_t w) { return -0.5f * neg2_log_u_word(w); }

// One Box-Muller pair: r = sqrt(-2 ln U1), (r cos 2 pi U2, r sin 2 pi U2).
// FAST, for the decision and weight kernels, whose FP32 values only steer the
// exact FP64 decision: r from the signed-word -log2 U1, i.e. every coordinate
// scaled by 1/sqrt(2 ln 2), a common factor that the projection onto the
// sphere removes (x^, t, S3 |x|^-3 and the mixture's ratios are invariant),
// and the angle from the signed word without the shift by half a turn.  The
// kernels that write rows for the caller keep the folded-word form and the
// unit scale, so that the rows' bits (and what is fitted to them, such as the
// learned proposal's networks) do not move with that choice.
template <bool FAST = false>
__device__ __forceinline__ void box_muller_f32(uint32_t w1, uint32_t w2, float &z0, float &z1)
{
    const float r = __builtin_amdgcn_sqrtf(FAST ? neg_log2_u_word_signed(w1)
                                                : neg2_log_u_word(w1));  // argument below 45
    if constexpr (FAST) {
        // w2 read as a signed integer: (s2 + 1/2) 2^-32 is U2 or U2 - 1, the same
        // angle in revolutions, in [-1/2, 1/2) as below
        const float rev = __builtin_fmaf((float)(int32_t)w2, 2.3283064365386963e-10f, 1.1641532182693481e-10f);
        z0 = r * __builtin_amdgcn_cosf(rev);
        z1 = r * __builtin_amdgcn_sinf(rev);
    } else {
        // U2 - 1/2 = (w2 - 2^31 + 1/2) 2^-32 in revolutions, centred on zero for
        // the hardware sin/cos; the signed integer w2 - 2^31 is formed exactly.
        const float rev = __builtin_fmaf((float)(int32_t)(w2 ^ 0x80000000u), 2.3283064365386963e-10f,
                                         1.1641532182693481e-10f);
        // sin/cos(2 pi (U2 - 1/2)) = -sin/-cos(2 pi U2)
        z0 = -r * __builtin_amdgcn_cosf(rev);
        z1 = -r * __builtin_amdgcn_sinf(rev);
    }
}

// ln(1 + y) for 0 <= y: the rounding of 1 + y is corrected to first order
// with the exact difference (1 + y) - 1 (an approximate reciprocal suffices).
__device__ __forceinline__ float log1p_f32(float y)
{
    const float u = 1.0f + y;
    const float den = u - 1.0f;
    const float lg = log2_hw(u) * 0.69314718055994531f;
    return den == 0.0f ? y : lg * (y * __builtin_amdgcn_rcpf(den));
}

__device__ __forceinline__ float xor32(float v) { return __shfl_xor(v, 32, 64); }

// ---------------------------------------------------------------------------
// Proposal generation: the K coordinates x of this lane's block (scaled by the
// proposal's standard deviations), |x|^-1, t = sum_k k^2 s_k of the projected
// point, and the acceptance word.  With NORMALIZE the coordinates are
// projected onto the sphere (x^ = x |x|^-1); otherwise the caller scales
// whatever it derives from x.  Both lanes of a proposal compute bitwise
// identical |x|^2 and t.  FAST selects the Box-Muller form (box_muller_f32):
// by default the signed-word form where the draw only feeds a decision or a
// weight, the folded-word form where rows are written.
// ---------------------------------------------------------------------------
template <int K, int PROP, bool NORMALIZE, bool FAST = !NORMALIZE>
__device__ __forceinline__ float gen_xhat(const DevPoint &P, uint64_t i, int half, float (&x)[K],
                                          float &t, uint32_t &w_acc)
{
    const uint32_t c0 = (uint32_t)i, c1 = (uint32_t)(i >> 32), c2 = P.point_id;
#pragma unroll
    for (int b = 0; b < K / 4; ++b) {
        uint4 w = philox4x32_10(c0, c1, c2, (uint32_t)(half * (K / 4) + b), P.key0, P.key1);
        box_muller_f32<FAST>(w.x, w.y, x[4 * b + 0], x[4 * b + 1]);
        box_muller_f32<FAST>(w.z, w.w, x[4 * b + 2], x[4 * b + 3]);
    }
    w_acc = philox4x32_10(c0, c1, c2, (uint32_t)(K / 2), P.key0, P.key1).x;
    if (PROP == PROP_SIGMA) {
#pragma unroll
        for (int j = 0; j < K; ++j) x[j] *= P.sig[j];
    }
    float r2 = 0.0f, tk = 0.0f;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const float sq = x[j] * x[j];
        r2 += sq;
        tk = __builtin_fmaf((float)((j + 1) * (j + 1)), sq, tk);
    }
    r2 = r2 + xor32(r2);
    tk = tk + xor32(tk);
    const float inv = __builtin_amdgcn_rsqf(r2);
    t = tk * (inv * inv);
    if (NORMALIZE) {
#pragma unroll
        for (int j = 0; j < K; ++j) x[j] *= inv;
    }
    return inv;
}

// ---------------------------------------------------------------------------
// Synthesis tables in LDS.
//   BF16: [T = K/8 grid tiles][S = K/8 k-steps][64 lanes][8] bf16, hi and lo;
//         lane l, tile t, step s holds Phi(block l/32, modes 8s+1..8s+8) at
//         grid point 32t + l%32.
//   FP32: [T][Q = K/4][64][4] floats; lane l holds Phi(block l/32, modes
//         4q+1..4q+4) at grid point 32t + l%32.
// ---------------------------------------------------------------------------
template <int K>
__host__ __device__ constexpr int bf16_table_bytes() { return (K / 8) * (K / 8) * kWave * 16; }
template <int K>
__host__ __device__ constexpr int f32_table_bytes() { return (K / 8) * (K / 4) * kWave * 16; }

// BF16 operands of this lane's coordinates: hi = RNE(x), lo = RNE(x - hi).
template <int K, int PREC>
__device__ __forceinline__ void split_bf16(const float (&x)[K], bf16x8 (&bh)[K / 8], bf16x8 (&bl)[K / 8])
{
#pragma unroll
    for (int s = 0; s < K / 8; ++s) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float v = x[8 * s + e];
            const __bf16 hv = (__bf16)v;
            bh[s][e] = hv;
            if constexpr (PREC == PREC_BF16X3) bl[s][e] = (__bf16)(v - (float)hv);
        }
    }
}

// Sum over this lane's grid values of u~^3 (u~ = unscaled synthesis), with
// the products in the requested arithmetic (FP32 reads x, BF16 reads bh/bl).
// The plain (dense) form; the kernels take it at K = 8, a single grid-tile
// group, and the half-period form below for K >= 16.
template <int K, int PREC>
__device__ __forceinline__ float cube_sum_ops(const float (&x)[K], const bf16x8 (&bh)[K / 8],
                                              const bf16x8 (&bl)[K / 8], const char *lds_hi,
                                              const char *lds_lo, int lane)
{
    float s3 = 0.0f;
    if constexpr (PREC == PREC_FP32) {
        const float4 *tab = reinterpret_cast<const float4 *>(lds_hi);
#pragma unroll
        for (int t = 0; t < K / 8; ++t) {
            f32x16 acc = {};
#pragma unroll
            for (int q = 0; q < K / 4; ++q) {
                float4 a = tab[(t * (K / 4) + q) * kWave + lane];
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, x[4 * q + 0], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, x[4 * q + 1], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, x[4 * q + 2], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, x[4 * q + 3], acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 16; ++v) s3 = __builtin_fmaf(acc[v] * acc[v], acc[v], s3);
        }
    } else {
        const bf16x8 *th = reinterpret_cast<const bf16x8 *>(lds_hi);
        const bf16x8 *tl = reinterpret_cast<const bf16x8 *>(lds_lo);
#pragma unroll
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
#pragma unroll
            for (int v = 0; v < 16; ++v) s3 = __builtin_fmaf(acc[v] * acc[v], acc[v], s3);
        }
    }
    return s3;
}

template <int K, int PREC>
__device__ __forceinline__ float synth_cube_sum(const float (&x)[K], const char *lds_hi,
                                                const char *lds_lo, int lane)
{
    bf16x8 bh[K / 8], bl[K / 8];
    if constexpr (PREC != PREC_FP32) split_bf16<K, PREC>(x, bh, bl);
    return cube_sum_ops<K, PREC>(x, bh, bl, lds_hi, lds_lo, lane);
}

// ---------------------------------------------------------------------------
// Half-period form of the synthesis (K >= 16).  Shifting the grid
// xi_j = -pi + 2 pi j/N by half a period (N/2 points, T/2 of the T = N/32
// grid tiles) multiplies mode k's cos and sin rows by (-1)^k.  With E and O
// the syntheses over the even and over the odd modes on grid tile t < T/2,
// tile t holds u~ = E + O and tile t + T/2 holds u~ = E - O, so that
//     u~(t)^3 + u~(t + T/2)^3 = 2 E (E^2 + 3 O^2):
// two products over half the modes each give both tiles, half the matrix
// work of the plain product for the same sum of cubes.
//   BF16 tables (hi, lo): fragment ((t * K/16 + s) * 2 + p) * 64 + l holds for
//   lane l the 8 entries Phi(block l/32, mode 16 s + 2 e + 2 - p) at grid
//   point 32 t + l%32 (p = 0 even modes, p = 1 odd modes), t < T/2, gathered
//   from the plain tables when a workgroup stages them.
//   FP32 table: the first T/2 grid tiles of the plain table (each FP32 matrix
//   instruction takes one mode; the parity selects the accumulator).
// ---------------------------------------------------------------------------
template <int K>
__host__ __device__ constexpr int eo_steps() { return K / 16; }  // k-steps of one parity = tile pairs

// bytes of one staged table (hi or lo)
template <int K, int PREC>
__host__ __device__ constexpr int eo_table_bytes()
{
    return (PREC == PREC_FP32 ? f32_table_bytes<K>() : bf16_table_bytes<K>()) / 2;
}

// Even-mode (p = 0) or odd-mode (p = 1) fragment from two consecutive k-step
// fragments a, b of the plain BF16 table (modes 8 s + 1 .. 8 s + 16): the even
// modes are their odd entries, the high halves of the 32-bit words.
__device__ __forceinline__ uint4 gather_parity(uint4 a, uint4 b, int p)
{
    if (p == 0)
        return make_uint4((a.x >> 16) | (a.y & 0xffff0000u), (a.z >> 16) | (a.w & 0xffff0000u),
                          (b.x >> 16) | (b.y & 0xffff0000u), (b.z >> 16) | (b.w & 0xffff0000u));
    return make_uint4((a.x & 0xffffu) | (a.y << 16), (a.z & 0xffffu) | (a.w << 16), (b.x & 0xffffu) | (b.y << 16),
                      (b.z & 0xffffu) | (b.w << 16));
}

// A workgroup of BLOCK threads permutes n_tiles row tiles of plain-layout
// BF16 fragments (tile t, k-step s: modes 8 s + 1 .. 8 s + 8) into the parity
// layout: fragment ((t * K/16 + s) * 2 + p) * 64 + l.
template <int K, int BLOCK>
__device__ __forceinline__ void stage_parity_frags(uint4 *dst, const uint4 *src, int n_tiles)
{
    constexpr int S = eo_steps<K>();
    const int n = n_tiles * (K / 8) * kWave;
    for (int v = threadIdx.x; v < n; v += BLOCK) {
        const int l = v % kWave, p = (v / kWave) % 2, s = (v / (2 * kWave)) % S, t = v / (2 * kWave * S);
        const int f = (t * (K / 8) + 2 * s) * kWave + l;  // plain fragment of k-step 2s
        dst[v] = gather_parity(src[f], src[f + kWave], p);
    }
}

// A workgroup of BLOCK threads stages the half-period tables: hi at lds, lo
// (BF16x3) at lds + eo_table_bytes.  The cube sums read tables whose odd-mode
// rows carry sqrt(3) (pair_cubes); the SIR power sums read the plain ones.
template <int K, int PREC, int BLOCK>
__device__ __forceinline__ void stage_eo_tables(char *lds, const void *phi_hi, const void *phi_lo)
{
    constexpr int tab = eo_table_bytes<K, PREC>();
    uint4 *d = reinterpret_cast<uint4 *>(lds);
    if constexpr (PREC == PREC_FP32) {
        const uint4 *s0 = reinterpret_cast<const uint4 *>(phi_hi);
        for (int v = threadIdx.x; v < tab / 16; v += BLOCK) d[v] = s0[v];
    } else {
        stage_parity_frags<K, BLOCK>(d, reinterpret_cast<const uint4 *>(phi_hi), eo_steps<K>());
        if constexpr (PREC == PREC_BF16X3)
            stage_parity_frags<K, BLOCK>(d + tab / 16, reinterpret_cast<const uint4 *>(phi_lo), eo_steps<K>());
    }
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// Two floats as packed BF16: hi = RNE(v), lo = RNE(v - hi) (the subtraction
// is exact: hi is v rounded to its top 16 bits).
__device__ __forceinline__ uint32_t pack_hi(float v0, float v1)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){v0, v1}, bf16x2_t));
}
__device__ __forceinline__ uint32_t pack_lo(float v0, float v1, uint32_t hi)
{
    const float h0 = __uint_as_float(hi << 16), h1 = __uint_as_float(hi & 0xffff0000u);
    return pack_hi(v0 - h0, v1 - h1);
}

// This lane's operands by parity (x[j] is the coordinate of mode j + 1):
// e*[s] entry e is mode 16 s + 2 e + 2, o*[s] entry e is mode 16 s + 2 e + 1.
// BF16 products fill eh and oh only.
template <int K, int PREC>
__device__ __forceinline__ void split_eo(const float (&x)[K], bf16x8 (&eh)[K / 16], bf16x8 (&el)[K / 16],
                                         bf16x8 (&oh)[K / 16], bf16x8 (&ol)[K / 16])
{
#pragma unroll
    for (int s = 0; s < K / 16; ++s) {
        u32x4_t weh, wel, woh, wol;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int j = 16 * s + 4 * w;
            weh[w] = pack_hi(x[j + 1], x[j + 3]);
            woh[w] = pack_hi(x[j], x[j + 2]);
            if constexpr (PREC == PREC_BF16X3) {
                wel[w] = pack_lo(x[j + 1], x[j + 3], weh[w]);
                wol[w] = pack_lo(x[j], x[j + 2], woh[w]);
            }
        }
        eh[s] = __builtin_bit_cast(bf16x8, weh);
        oh[s] = __builtin_bit_cast(bf16x8, woh);
        if constexpr (PREC == PREC_BF16X3) {
            el[s] = __builtin_bit_cast(bf16x8, wel);
            ol[s] = __builtin_bit_cast(bf16x8, wol);
        }
    }
}

// hi operands only (BF16 products)
template <int K>
__device__ __forceinline__ void split_eo_hi(const float (&x)[K], bf16x8 (&eh)[K / 16], bf16x8 (&oh)[K / 16])
{
#pragma unroll
    for (int s = 0; s < K / 16; ++s) {
        u32x4_t weh, woh;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int j = 16 * s + 4 * w;
            weh[w] = pack_hi(x[j + 1], x[j + 3]);
            woh[w] = pack_hi(x[j], x[j + 2]);
        }
        eh[s] = __builtin_bit_cast(bf16x8, weh);
        oh[s] = __builtin_bit_cast(bf16x8, woh);
    }
}

// sum over the pair's grid values of u~^3 = 2 E (E^2 + 3 O^2), elementwise,
// from co = sqrt(3) O: the odd-mode rows of the tables these sums read carry
// the factor sqrt(3), which saves a product per grid value (the factor 2 is
// applied by the caller)
__device__ __forceinline__ float pair_cubes(const f32x16 &ce, const f32x16 &co, float s)
{
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const float e = ce[v], o = co[v];
        const float q = __builtin_fmaf(o, o, e * e);
        s = __builtin_fmaf(e, q, s);
    }
    return s;
}

// S3 over this lane's grid values in the half-period form, FP32 products; G
// tile pairs per group have their accumulators live together.  The tables are
// the S3 tables: odd-mode rows scaled by sqrt(3) (pair_cubes).
template <int K, int G>
__device__ __forceinline__ float cube_sum_eo_f32(const float (&x)[K], const char *lds, int lane)
{
    constexpr int P = eo_steps<K>();
    const float4 *tab = reinterpret_cast<const float4 *>(lds);
    float s3 = 0.0f;
#pragma unroll 1
    for (int g = 0; g < P; g += G) {
        f32x16 ce[G], co[G];
#pragma unroll
        for (int u = 0; u < G; ++u) ce[u] = co[u] = f32x16{};
#pragma unroll
        for (int q = 0; q < K / 4; ++q)
#pragma unroll
            for (int u = 0; u < G; ++u) {
                // entries 0..3: modes 4q+1 (odd), 4q+2 (even), 4q+3 (odd), 4q+4 (even)
                const float4 a = tab[((g + u) * (K / 4) + q) * kWave + lane];
                co[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, x[4 * q + 0], co[u], 0, 0, 0);
                ce[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, x[4 * q + 1], ce[u], 0, 0, 0);
                co[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, x[4 * q + 2], co[u], 0, 0, 0);
                ce[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, x[4 * q + 3], ce[u], 0, 0, 0);
            }
#pragma unroll
        for (int u = 0; u < G; ++u) s3 = pair_cubes(ce[u], co[u], s3);
    }
    return 2.0f * s3;
}

// The same with BF16 (hi) or BF16x3 (hi/lo) products from the split operands;
// the lo operands el, ol are read for BF16x3 only (null for BF16).
template <int K, int PREC, int G>
__device__ __forceinline__ float cube_sum_eo_bf16(const bf16x8 (&eh)[K / 16], const bf16x8 *el,
                                                  const bf16x8 (&oh)[K / 16], const bf16x8 *ol,
                                                  const char *lds_hi, const char *lds_lo, int lane)
{
    constexpr int P = eo_steps<K>(), S = eo_steps<K>();
    const bf16x8 *th = reinterpret_cast<const bf16x8 *>(lds_hi);
    const bf16x8 *tl = reinterpret_cast<const bf16x8 *>(lds_lo);
    float s3 = 0.0f;
#pragma unroll 1
    for (int g = 0; g < P; g += G) {
        f32x16 ce[G], co[G];
#pragma unroll
        for (int u = 0; u < G; ++u) ce[u] = co[u] = f32x16{};
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int idx = ((g + u) * S + s) * 2 * kWave + lane;
                const bf16x8 aeh = th[idx], aoh = th[idx + kWave];
                if constexpr (PREC == PREC_BF16X3) {
                    const bf16x8 ael = tl[idx], aol = tl[idx + kWave];
                    ce[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ael, eh[s], ce[u], 0, 0, 0);
                    co[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aol, oh[s], co[u], 0, 0, 0);
                    ce[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aeh, el[s], ce[u], 0, 0, 0);
                    co[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aoh, ol[s], co[u], 0, 0, 0);
                }
                ce[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aeh, eh[s], ce[u], 0, 0, 0);
                co[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aoh, oh[s], co[u], 0, 0, 0);
            }
#pragma unroll
        for (int u = 0; u < G; ++u) s3 = pair_cubes(ce[u], co[u], s3);
    }
    return 2.0f * s3;
}

// S3 of coordinates x in the half-period form with G tile pairs per group.
template <int K, int PREC, int G>
__device__ __forceinline__ float eo_cube_sum(const float (&x)[K], const char *lds_hi, const char *lds_lo, int lane)
{
    if constexpr (PREC == PREC_FP32) {
        return cube_sum_eo_f32<K, G>(x, lds_hi, lane);
    } else {
        constexpr int S = eo_steps<K>();
        bf16x8 eh[S], oh[S];
        if constexpr (PREC == PREC_BF16X3) {
            bf16x8 el[S], ol[S];
            split_eo<K, PREC>(x, eh, el, oh, ol);
            return cube_sum_eo_bf16<K, PREC, G>(eh, el, oh, ol, lds_hi, lds_lo, lane);
        } else {
            split_eo_hi<K>(x, eh, oh);
            return cube_sum_eo_bf16<K, PREC, G>(eh, nullptr, oh, nullptr, lds_hi, lds_lo, lane);
        }
    }
}

// log a = log f/(M g) in FP32 from t and S3 = sum_j u~_j^3 (both lanes identical).
template <int PROP>
__device__ __forceinline__ float log_a_f32(const DevPoint &P, float t, float s3)
{
    float lf = __builtin_fmaf(P.neg_bp_K2, t, P.c3coef * s3);
    if (PROP == PROP_SIGMA) lf = __builtin_fmaf(P.Kf, log1p_f32(P.g_coef * t), lf);
    return lf - P.log_M;
}

// Order-preserving map float -> uint32 for atomicMax.
__device__ __forceinline__ unsigned int float_key(float f)
{
    unsigned int u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Thresholds of the statistics in units of u~ = u / sqrt(2 E0/pi): 2 sigma and
// 4 sigma, sigma = sqrt(E0/pi), are u~ = sqrt 2 and 2 sqrt 2.
constexpr float kTwoSigmaT = 1.41421356237309515f;
constexpr float kFourSigmaT = 2.82842712474619031f;

// The better of two peaks (float_key of the value, proposal index): the larger
// value, the lower index among equal values; key 0 stands for none.
__device__ __forceinline__ void peak_merge(unsigned int &key, unsigned long long &idx, unsigned int k2,
                                           unsigned long long i2)
{
    if (k2 > key || (k2 == key && k2 != 0u && i2 < idx)) {
        key = k2;
        idx = i2;
    }
}
// The peak of the wave, in every lane (the merge is a total order).
__device__ __forceinline__ void wave_peak(unsigned int &key, unsigned long long &idx)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned int k2 = __shfl_xor(key, o, 64);
        const unsigned long long i2 = __shfl_xor(idx, o, 64);
        peak_merge(key, idx, k2, i2);
    }
}

__device__ __forceinline__ unsigned long long pack_defer(int p, uint64_t i)
{
    return ((unsigned long long)p << 40) | (unsigned long long)i;
}

// log f = -beta'/(E0 K^2) (H2 - c H3) in FP64 at a point x of the sphere with
// t = sum k^2 s_k: H2 = E0 t by Parseval and H3 by the double sum over the
// triads k + (n - k) = n (Sec. IV.A).
__device__ inline double log_f_fp64(int K, double E0, double beta_p, double c32, const double *x, double t)
{
    const double pi = 3.14159265358979323846;
    const double s = sqrt(E0 / (2.0 * pi));
    double tri = 0.0;
    for (int n = 2; n <= K; ++n) {
        double in_re = 0.0, in_im = 0.0;
        for (int k = 1; k < n; ++k) {
            const double pr = s * x[k - 1], pi_ = -s * x[K + k - 1];
            const double qr = s * x[n - k - 1], qi = -s * x[K + n - k - 1];
            in_re += pr * qr - pi_ * qi;
            in_im += pr * qi + pi_ * qr;
        }
        tri += (s * x[n - 1]) * in_re + (-s * x[K + n - 1]) * in_im;
    }
    const double H3 = 2.0 * pi * tri;
    const double H2 = E0 * t;
    return -(beta_p / (E0 * (double)K * K) * (H2 - c32 * H3));
}

// ---------------------------------------------------------------------------
// Learned mixture proposal
// ---------------------------------------------------------------------------
// Component of a proposal from its component word: -1 (g_Sigma) when w < E,
// else j = (w - E) div B, formed in integers (one FP32 estimate, corrected
// by one step: the estimate is within 1 of the quotient).
__device__ __forceinline__ int mix_component(const DevMix &M, uint32_t w)
{
    const uint32_t d = w - M.E;
    uint32_t j = (uint32_t)((float)d * M.invB);
    j = j > (uint32_t)(kMixS - 1) ? (uint32_t)(kMixS - 1) : j;
    const uint32_t prod = j * M.B;
    if (prod > d) --j;
    else if (d - prod >= M.B) ++j;
    return w < M.E ? -1 : (int)j;
}

// Draw of proposal i from q_mix: this lane's K coordinates of X (words
// 0..2K-1 as for the paper's proposal, word 2K the acceptance word, 2K+1 the
// component word, 2K+2 and 2K+3 the pair eta), |X|^-1, t of the projected
// point and Qa = sum over this proposal of a_c X_c^2 (unprojected).  rv
// points to the RV table of the point (LDS or global memory).  FAST as for
// gen_xhat.
template <int K, bool NORMALIZE, bool FAST = !NORMALIZE>
__device__ __forceinline__ float gen_x_mix(const DevPoint &P, const DevMix &M, const float *rv, uint64_t i,
                                           int half, float (&x)[K], float &t, float &Qa, uint32_t &w_acc)
{
    const uint32_t c0 = (uint32_t)i, c1 = (uint32_t)(i >> 32), c2 = P.point_id;
#pragma unroll
    for (int b = 0; b < K / 4; ++b) {
        uint4 w = philox4x32_10(c0, c1, c2, (uint32_t)(half * (K / 4) + b), P.key0, P.key1);
        box_muller_f32<FAST>(w.x, w.y, x[4 * b + 0], x[4 * b + 1]);
        box_muller_f32<FAST>(w.z, w.w, x[4 * b + 2], x[4 * b + 3]);
    }
    const uint4 wl = philox4x32_10(c0, c1, c2, (uint32_t)(K / 2), P.key0, P.key1);
    w_acc = wl.x;
    const int comp = mix_component(M, wl.y);
    const bool def = comp < 0;
    float e0, e1;
    box_muller_f32<FAST>(wl.z, wl.w, e0, e1);
    e0 = def ? 0.0f : e0;
    e1 = def ? 0.0f : e1;
    const float2 *row = reinterpret_cast<const float2 *>(rv + (2 * (def ? 0 : comp) + half) * (2 * K + 2));
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const float sc = def ? P.sig[j] : M.sqd[j];
        const float2 v = row[j];
        x[j] = __builtin_fmaf(v.x, e0, __builtin_fmaf(v.y, e1, sc * x[j]));
    }
    float r2 = 0.0f, tk = 0.0f, qa = 0.0f;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const float sq = x[j] * x[j];
        r2 += sq;
        tk = __builtin_fmaf((float)((j + 1) * (j + 1)), sq, tk);
        qa = __builtin_fmaf(M.a[j], sq, qa);
    }
    r2 = r2 + xor32(r2);
    tk = tk + xor32(tk);
    Qa = qa + xor32(qa);
    const float inv = __builtin_amdgcn_rsqf(r2);
    t = tk * (inv * inv);
    if (NORMALIZE) {
#pragma unroll
        for (int j = 0; j < K; ++j) x[j] *= inv;
    }
    return inv;
}

// z = (R_j A V C^T)^T X for the S shifts on the matrix cores (C^T C = G^-1, so
// that y_j^T G^-1 y_j = |z_j|^2): row tile q holds rank index q, row j the
// shift, column the proposal (the B operand layout).  Row tiles share their row
// order, so y0[v] and y1[v] are the two entries of one shift's z.
template <int K, int PREC>
__device__ __forceinline__ void mix_y(const float (&x)[K], const bf16x8 (&bh)[K / 8], const bf16x8 (&bl)[K / 8],
                                      const char *yt_hi, const char *yt_lo, int lane, f32x16 &y0, f32x16 &y1)
{
    if constexpr (PREC == PREC_FP32) {
        const float4 *tab = reinterpret_cast<const float4 *>(yt_hi);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            f32x16 acc = {};
#pragma unroll
            for (int q = 0; q < K / 4; ++q) {
                float4 a = tab[(t * (K / 4) + q) * kWave + lane];
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, x[4 * q + 0], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, x[4 * q + 1], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, x[4 * q + 2], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, x[4 * q + 3], acc, 0, 0, 0);
            }
            if (t == 0) y0 = acc; else y1 = acc;
        }
    } else {
        const bf16x8 *th = reinterpret_cast<const bf16x8 *>(yt_hi);
        const bf16x8 *tl = reinterpret_cast<const bf16x8 *>(yt_lo);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
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
            if (t == 0) y0 = acc; else y1 = acc;
        }
    }
}

// The same products from the parity-split operands (split_eo) against the
// y tables staged in the parity layout (stage_parity_frags, 2 row tiles); the
// two row tiles accumulate as independent chains.  FP32 reads x as mix_y.
template <int K, int PREC>
__device__ __forceinline__ void mix_y_eo(const float (&x)[K], const bf16x8 (&eh)[K / 16], const bf16x8 *el,
                                         const bf16x8 (&oh)[K / 16], const bf16x8 *ol, const char *yt_hi,
                                         const char *yt_lo, int lane, f32x16 &y0, f32x16 &y1)
{
    if constexpr (PREC == PREC_FP32) {
        bf16x8 bh[K / 8], bl[K / 8];
        mix_y<K, PREC>(x, bh, bl, yt_hi, yt_lo, lane, y0, y1);
    } else {
        constexpr int S = eo_steps<K>();
        const bf16x8 *th = reinterpret_cast<const bf16x8 *>(yt_hi);
        const bf16x8 *tl = reinterpret_cast<const bf16x8 *>(yt_lo);
        f32x16 acc[2] = {f32x16{}, f32x16{}};
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int idx = ((t * S + s) * 2 + p) * kWave + lane;
                    const bf16x8 &bh = p == 0 ? eh[s] : oh[s];
                    const bf16x8 ah = th[idx];
                    if constexpr (PREC == PREC_BF16X3) {
                        const bf16x8 &bl = p == 0 ? el[s] : ol[s];
                        const bf16x8 al = tl[idx];
                        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[t], 0, 0, 0);
                        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[t], 0, 0, 0);
                    }
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[t], 0, 0, 0);
                }
        y0 = acc[0];
        y1 = acc[1];
    }
}

// log q_mix in FP32 from the shifts' z, Qa = X^T A X (both unprojected: the
// ratios r_j = qf_j/Q = 1 - |z_j|^2/Qa are scale free), |X|^-2 and t.
//   ln q_net + ln(1 - eps) = c_net - K ln(Qa |X|^-2) + ln sum_j r_j^-K,
//   ln(eps g_Sigma) = c_g - K ln(1 + alpha beta' t/K^3).
// The sum is taken relative to the smallest r_j of the proposal (all terms
// <= 1, the largest exactly 1).  Both lanes of a proposal return the same.
__device__ __forceinline__ float mix_log_q_f32(const DevPoint &P, const DevMix &M, const f32x16 &y0,
                                               const f32x16 &y1, float Qa, float inv2, float t, float Kf)
{
    const float invQ = __builtin_amdgcn_rcpf(Qa);
    float l[16];
    float lmin = INFINITY;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const float a0 = y0[v], a1 = y1[v];
        const float quad = __builtin_fmaf(a0, a0, a1 * a1);
        const float r = fmaxf(__builtin_fmaf(-quad, invQ, 1.0f), 1e-30f);
        l[v] = log2_hw(r);
        lmin = fminf(lmin, l[v]);
    }
    lmin = fminf(lmin, xor32(lmin));
    // K (lmin - l) as one FMA: K is a power of two (8, 16, 32), so K lmin is
    // exact and the FMA rounds the same exact value as the difference scaled
    const float klmin = Kf * lmin;
    float sum = __builtin_amdgcn_exp2f(__builtin_fmaf(-Kf, l[0], klmin));
#pragma unroll
    for (int v = 1; v < 16; ++v) sum += __builtin_amdgcn_exp2f(__builtin_fmaf(-Kf, l[v], klmin));
    sum = sum + xor32(sum);
    const float ln2 = 0.69314718055994531f;
    const float LN = M.c_net + ln2 * (log2_hw(sum) - Kf * (lmin + log2_hw(Qa * inv2)));
    const float LG = M.c_g - Kf * log1p_f32(P.g_coef * t);
    const float hi = fmaxf(LN, LG);
    return hi + log1p_f32(__builtin_amdgcn_exp2f(-fabsf(LN - LG) * 1.4426950408889634f));
}

}  // namespace tkdv
