// The standalone spectral-to-grid synthesis: rows of x^ in HBM -> the sum of
// the cubes of the grid values of each row, S3 = sum_j u~_j^3 (u~ = Phi^T x^
// unscaled, N = 4K grid points; H3 of Eq. (H3H2) is (pi/(3N)) (2 E0/pi)^{3/2}
// S3), with the products on the matrix cores in FP32, BF16 or BF16x3.
//
// Half-period symmetry.  Shifting the grid xi_j = -pi + 2 pi j/N by half a
// period (N/2 points, T/2 of the T = N/32 grid tiles) multiplies mode k's cos
// and sin rows by (-1)^k.  With E and O the syntheses over the even and over
// the odd modes on grid tile t < T/2, tile t holds u~ = E + O and tile
// t + T/2 holds u~ = E - O, so that
//     u~(t)^3 + u~(t + T/2)^3 = 2 E (E^2 + 3 O^2).
// Two products over half the modes each give both tiles: half the matrix
// work of the plain product Phi^T x^ for the same S3, and no sign flips.
// K = 8 (a single grid tile) takes the plain product.
#include <hip/hip_runtime.h>

#include "tkdv_device.h"
#include "tkdv_internal.h"
#include "tkdv_kernels.h"

namespace tkdv {
namespace {

// Grid-tile pairs (T/2) and the k-steps of one parity (8 modes per block).
template <int K>
constexpr int eo_pairs() { return K / 16; }
template <int K>
constexpr int eo_steps() { return K / 16; }
// Tile pairs whose accumulators are live together (consecutive matrix
// instructions then update different accumulators): two at K = 32, one at
// K = 64, where four waves per SIMD leave 128 registers a lane.
template <int K>
constexpr int eo_group() { return K == 32 ? 2 : 1; }

// Bytes of one table (hi or lo) in LDS.  BF16, K >= 16: the even/odd form,
// fragment ((t * eo_steps + s) * 2 + p) * 64 + l holds for lane l the 8
// entries Phi(block l/32, mode 16 s + 2 e + 2 - p) at grid point 32 t + l%32
// (p = 0 even modes, p = 1 odd modes), t < T/2.  FP32, K >= 16: the first T/2
// grid tiles of the plain FP32 table (each MFMA takes one mode, so the parity
// only selects the accumulator).  K = 8: the whole plain table.
template <int K, int PREC>
constexpr int synth_tab_bytes()
{
    constexpr int full = PREC == PREC_FP32 ? f32_table_bytes<K>() : bf16_table_bytes<K>();
    return K == 8 ? full : full / 2;
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

template <int K, int PREC, int BLOCK>
__device__ __forceinline__ void stage_tables(char *lds, const void *phi_hi, const void *phi_lo)
{
    constexpr int tab = synth_tab_bytes<K, PREC>();
    uint4 *d = reinterpret_cast<uint4 *>(lds);
    if constexpr (K == 8 || PREC == PREC_FP32) {
        const uint4 *s0 = reinterpret_cast<const uint4 *>(phi_hi);
        for (int v = threadIdx.x; v < tab / 16; v += BLOCK) d[v] = s0[v];
        if constexpr (PREC == PREC_BF16X3) {
            const uint4 *s1 = reinterpret_cast<const uint4 *>(phi_lo);
            for (int v = threadIdx.x; v < tab / 16; v += BLOCK) d[tab / 16 + v] = s1[v];
        }
    } else {
        constexpr int S = eo_steps<K>();
        for (int part = 0; part < (PREC == PREC_BF16X3 ? 2 : 1); ++part) {
            const uint4 *src = reinterpret_cast<const uint4 *>(part == 0 ? phi_hi : phi_lo);
            uint4 *dst = d + part * (tab / 16);
            for (int v = threadIdx.x; v < tab / 16; v += BLOCK) {
                const int l = v % kWave, p = (v / kWave) % 2, s = (v / (2 * kWave)) % S, t = v / (2 * kWave * S);
                const int f = (t * (K / 8) + 2 * s) * kWave + l;  // plain fragment of k-step 2s
                dst[v] = gather_parity(src[f], src[f + kWave], p);
            }
        }
    }
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));  // rows in registers (native vectors)
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

// hi operands only (BF16 products), as split_eo below
template <int K>
__device__ __forceinline__ void split_eo_hi(const f32x4_t (&r)[K / 4], bf16x8 (&eh)[K / 16], bf16x8 (&oh)[K / 16])
{
#pragma unroll
    for (int s = 0; s < K / 16; ++s) {
        const u32x4_t weh = {pack_hi(r[4 * s].y, r[4 * s].w), pack_hi(r[4 * s + 1].y, r[4 * s + 1].w),
                             pack_hi(r[4 * s + 2].y, r[4 * s + 2].w), pack_hi(r[4 * s + 3].y, r[4 * s + 3].w)};
        const u32x4_t woh = {pack_hi(r[4 * s].x, r[4 * s].z), pack_hi(r[4 * s + 1].x, r[4 * s + 1].z),
                             pack_hi(r[4 * s + 2].x, r[4 * s + 2].z), pack_hi(r[4 * s + 3].x, r[4 * s + 3].z)};
        eh[s] = __builtin_bit_cast(bf16x8, weh);
        oh[s] = __builtin_bit_cast(bf16x8, woh);
    }
}

// This lane's operands by parity from its K coordinates r (r[q] = x[4q..4q+3],
// x[j] the coordinate of mode j + 1): e*[s] entry e is mode 16 s + 2 e + 2,
// o*[s] entry e is mode 16 s + 2 e + 1; 32-bit word w of k-step s pairs the
// coordinates of r[4 s + w] (.y, .w even modes, .x, .z odd modes).
template <int K, int PREC>
__device__ __forceinline__ void split_eo(const f32x4_t (&r)[K / 4], bf16x8 (&eh)[K / 16], bf16x8 (&el)[K / 16],
                                         bf16x8 (&oh)[K / 16], bf16x8 (&ol)[K / 16])
{
#pragma unroll
    for (int s = 0; s < K / 16; ++s) {
        u32x4_t weh, wel, woh, wol;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const f32x4_t v = r[4 * s + w];
            weh[w] = pack_hi(v.y, v.w);
            woh[w] = pack_hi(v.x, v.z);
            if constexpr (PREC == PREC_BF16X3) {
                wel[w] = pack_lo(v.y, v.w, weh[w]);
                wol[w] = pack_lo(v.x, v.z, woh[w]);
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

// sum over the pair's grid values of u~^3 = 2 E (E^2 + 3 O^2), elementwise
__device__ __forceinline__ float pair_cubes(const f32x16 &ce, const f32x16 &co, float s)
{
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const float e = ce[v], o = co[v];
        const float q = __builtin_fmaf(3.0f * o, o, e * e);
        s = __builtin_fmaf(e, q, s);
    }
    return s;
}

// S3 over this lane's grid values (K >= 16), even/odd form, FP32 products.
template <int K>
__device__ __forceinline__ float cube_sum_eo_f32(const float (&x)[K], const char *lds, int lane)
{
    constexpr int P = eo_pairs<K>(), G = eo_group<K>();
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

// The same with BF16 (hi) or BF16x3 (hi/lo) products from the split operands.
template <int K, int PREC>
__device__ __forceinline__ float cube_sum_eo_bf16(const bf16x8 (&eh)[K / 16], const bf16x8 (&el)[K / 16],
                                                  const bf16x8 (&oh)[K / 16], const bf16x8 (&ol)[K / 16],
                                                  const char *lds_hi, const char *lds_lo, int lane)
{
    constexpr int P = eo_pairs<K>(), S = eo_steps<K>(), G = eo_group<K>();
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

// Persistent workgroups keep the tables in LDS and loop over 32-row tiles;
// lanes p / p + 32 read the cos / sin half of row p (K contiguous floats)
// straight into the operand registers.
template <int K, int PREC, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_synth(const float *__restrict__ xhat, unsigned long long n,
                                                 float *__restrict__ s3_out, const void *phi_hi,
                                                 const void *phi_lo)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    constexpr int tab = synth_tab_bytes<K, PREC>();
    stage_tables<K, PREC, BLOCK>(lds, phi_hi, phi_lo);
    __syncthreads();
    const int lane = threadIdx.x & 63, half = lane >> 5, pl = lane & 31;
    const unsigned long long n_tiles = (n + kTile - 1) / kTile;
    const unsigned long long waves = (unsigned long long)gridDim.x * (BLOCK / kWave);
    unsigned long long tile = (unsigned long long)blockIdx.x * (BLOCK / kWave) + (threadIdx.x >> 6);
    // K < 64: rows of the next tile are loaded while the current tile is on the
    // matrix cores.  BF16 products (K >= 16): the current rows are split into
    // operands first, so the loads of the next rows reuse their registers
    // (issued unconditionally: past the last tile they read row 0 again).
    // FP32 and K = 8 keep the rows as operands and prefetch where the register
    // budget allows it (not beside the four live K = 32 FP32 accumulators).
    // K = 64 runs four waves per SIMD instead, which hide the loads.
    constexpr bool split_first = K >= 16 && PREC != PREC_FP32;
    constexpr bool prefetch = K < 64 && (split_first || !(K == 32 && PREC == PREC_FP32));
    f32x4_t nxt[K / 4];
    auto load_tile = [&](unsigned long long tl) {
        const unsigned long long row = tl * kTile + pl;
        const unsigned long long r = (tl < n_tiles && row < n) ? row : 0ull;
        const f32x4_t *src = reinterpret_cast<const f32x4_t *>(xhat + r * (2 * K) + half * K);
#pragma unroll
        for (int q = 0; q < K / 4; ++q) nxt[q] = src[q];
    };
    if (prefetch && tile < n_tiles) load_tile(tile);
    for (; tile < n_tiles; tile += waves) {
        if (!prefetch) load_tile(tile);
        const unsigned long long row = tile * kTile + pl;
        const bool valid = row < n;
        float s3l;
        if constexpr (split_first) {
            constexpr int S = eo_steps<K>();
            bf16x8 eh[S], oh[S];
            if constexpr (PREC == PREC_BF16X3) {
                bf16x8 el[S], ol[S];
                split_eo<K, PREC>(nxt, eh, el, oh, ol);
                __builtin_amdgcn_sched_barrier(0);
                if (prefetch) load_tile(tile + waves);
                s3l = cube_sum_eo_bf16<K, PREC>(eh, el, oh, ol, lds, lds + tab, lane);
            } else {  // no lo operands: the hi arrays stand in, unread
                split_eo_hi<K>(nxt, eh, oh);
                __builtin_amdgcn_sched_barrier(0);
                if (prefetch) load_tile(tile + waves);
                s3l = cube_sum_eo_bf16<K, PREC>(eh, eh, oh, oh, lds, lds + tab, lane);
            }
        } else {
            float x[K];
#pragma unroll
            for (int q = 0; q < K / 4; ++q) {
                x[4 * q + 0] = nxt[q].x;
                x[4 * q + 1] = nxt[q].y;
                x[4 * q + 2] = nxt[q].z;
                x[4 * q + 3] = nxt[q].w;
            }
            if (prefetch && tile + waves < n_tiles) load_tile(tile + waves);
            if constexpr (K == 8) {
                bf16x8 bh[1], bl[1];
                if constexpr (PREC != PREC_FP32) split_bf16<K, PREC>(x, bh, bl);
                s3l = cube_sum_ops<K, PREC>(x, bh, bl, lds, lds + tab, lane);
            } else {
                s3l = cube_sum_eo_f32<K>(x, lds, lane);
            }
        }
        const float s3 = s3l + xor32(s3l);
        if (valid && half == 0) s3_out[row] = s3;
    }
}

// Workgroup size: 8 waves; 16 at K = 64 (one workgroup and one copy of the
// 64 KB BF16x3 tables per CU, four waves per SIMD).
template <int K>
constexpr int synth_block() { return K == 64 ? 2 * kSynthBlock : kSynthBlock; }

template <int K, int PREC>
constexpr int synth_lds_bytes()
{
    return (PREC == PREC_BF16X3 ? 2 : 1) * synth_tab_bytes<K, PREC>();
}

template <int K, int PREC>
hipError_t launch_synth_t(const float *xhat, unsigned long long n, float *s3, const void *phi_hi,
                          const void *phi_lo, int n_cu, hipStream_t st, hipEvent_t ev_start, int *grid_out,
                          int *block_out)
{
    constexpr int lds = synth_lds_bytes<K, PREC>();
    constexpr int B = synth_block<K>();
    auto kern = k_synth<K, PREC, B>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, B, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    const unsigned long long tiles = (n + kTile - 1) / kTile;
    unsigned long long grid = (unsigned long long)per_cu * n_cu;
    const unsigned long long want = (tiles + B / kWave - 1) / (B / kWave);
    if (want < grid) grid = want;
    if (grid < 1) grid = 1;
    if (grid_out) *grid_out = (int)grid;
    if (block_out) *block_out = B;
    if (ev_start) {
        e = hipEventRecord(ev_start, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(B), lds, st, xhat, n, s3, phi_hi, phi_lo);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_synth(int K, int prec, const float *xhat, unsigned long long n, float *s3, const void *phi_hi,
                        const void *phi_lo, int n_cu, hipStream_t st, hipEvent_t ev_start, int *grid_out,
                        int *block_out)
{
#define TKDV_DISPATCH_S(KK, PR)                                                                         \
    if (K == KK && prec == PR)                                                                          \
        return launch_synth_t<KK, PR>(xhat, n, s3, phi_hi, phi_lo, n_cu, st, ev_start, grid_out, block_out);
    TKDV_DISPATCH_S(8, PREC_FP32) TKDV_DISPATCH_S(8, PREC_BF16) TKDV_DISPATCH_S(8, PREC_BF16X3)
    TKDV_DISPATCH_S(16, PREC_FP32) TKDV_DISPATCH_S(16, PREC_BF16) TKDV_DISPATCH_S(16, PREC_BF16X3)
    TKDV_DISPATCH_S(32, PREC_FP32) TKDV_DISPATCH_S(32, PREC_BF16) TKDV_DISPATCH_S(32, PREC_BF16X3)
    TKDV_DISPATCH_S(64, PREC_FP32) TKDV_DISPATCH_S(64, PREC_BF16) TKDV_DISPATCH_S(64, PREC_BF16X3)
#undef TKDV_DISPATCH_S
    return hipErrorInvalidValue;
}

}  // namespace tkdv
