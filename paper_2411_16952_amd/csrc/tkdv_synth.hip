// The standalone spectral-to-grid synthesis: rows of x^ in HBM -> the sum of
// the cubes of the grid values of each row, S3 = sum_j u~_j^3 (u~ = Phi^T x^
// unscaled, N = 4K grid points; H3 of Eq. (H3H2) is (pi/(3N)) (2 E0/pi)^{3/2}
// S3), with the products on the matrix cores in FP32, BF16 or BF16x3.  K >= 16
// takes the half-period form of the synthesis (tkdv_device.h: half the matrix
// work of the plain product); K = 8 (a single grid tile) the plain product.
#include <hip/hip_runtime.h>

#include "tkdv_device.h"
#include "tkdv_internal.h"
#include "tkdv_kernels.h"

namespace tkdv {
namespace {

// Tile pairs whose accumulators are live together (consecutive matrix
// instructions then update different accumulators): two at K = 32, one at
// K = 64, where four waves per SIMD leave 128 registers a lane.
template <int K>
constexpr int synth_group() { return K == 32 ? 2 : 1; }

// Bytes of one staged table (hi or lo): the half-period tables for K >= 16,
// the whole plain table at K = 8.
template <int K, int PREC>
constexpr int synth_tab_bytes()
{
    constexpr int full = PREC == PREC_FP32 ? f32_table_bytes<K>() : bf16_table_bytes<K>();
    return K == 8 ? full : eo_table_bytes<K, PREC>();
}

template <int K, int PREC, int BLOCK>
__device__ __forceinline__ void stage_tables(char *lds, const void *phi_hi, const void *phi_lo)
{
    if constexpr (K == 8) {
        constexpr int tab = synth_tab_bytes<K, PREC>();
        uint4 *d = reinterpret_cast<uint4 *>(lds);
        const uint4 *s0 = reinterpret_cast<const uint4 *>(phi_hi);
        for (int v = threadIdx.x; v < tab / 16; v += BLOCK) d[v] = s0[v];
        if constexpr (PREC == PREC_BF16X3) {
            const uint4 *s1 = reinterpret_cast<const uint4 *>(phi_lo);
            for (int v = threadIdx.x; v < tab / 16; v += BLOCK) d[tab / 16 + v] = s1[v];
        }
    } else {
        stage_eo_tables<K, PREC, BLOCK>(lds, phi_hi, phi_lo);
    }
}

typedef float f32x4_t __attribute__((ext_vector_type(4)));  // rows in registers (native vectors)

// split_eo_hi straight from the loaded row vectors r[q] = x[4q .. 4q+3] (the
// BF16 path; going through a float array left stack copies of it)
template <int K>
__device__ __forceinline__ void split_eo_hi_rows(const f32x4_t (&r)[K / 4], bf16x8 (&eh)[K / 16], bf16x8 (&oh)[K / 16])
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
                float x[K];
#pragma unroll
                for (int q = 0; q < K / 4; ++q) {
                    x[4 * q + 0] = nxt[q].x;
                    x[4 * q + 1] = nxt[q].y;
                    x[4 * q + 2] = nxt[q].z;
                    x[4 * q + 3] = nxt[q].w;
                }
                bf16x8 el[S], ol[S];
                split_eo<K, PREC>(x, eh, el, oh, ol);
                __builtin_amdgcn_sched_barrier(0);
                if (prefetch) load_tile(tile + waves);
                s3l = cube_sum_eo_bf16<K, PREC, synth_group<K>()>(eh, el, oh, ol, lds, lds + tab, lane);
            } else {
                split_eo_hi_rows<K>(nxt, eh, oh);
                __builtin_amdgcn_sched_barrier(0);
                if (prefetch) load_tile(tile + waves);
                s3l = cube_sum_eo_bf16<K, PREC, synth_group<K>()>(eh, nullptr, oh, nullptr, lds, lds + tab, lane);
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
                s3l = cube_sum_eo_f32<K, synth_group<K>()>(x, lds, lane);
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
