// Extreme wave fields among stored samples (Sec. V, the search of individual
// samples for the largest surface displacement):
//   k_grid_max   per row x^: u on the N = 4K grid (u = amp Phi^T x^, FP32
//                matrix products from the FP32 synthesis tables in LDS), its
//                maximum, the first grid index attaining it, and the count of
//                rows whose maximum exceeds a threshold (K <= 32);
//   k_grid_max_q the same in the quarter-period form (K = 64, 128);
//   k_key_hist   one pass of an exact radix select over order-preserving keys
//                of the maxima (8 bits per pass, restricted to a key prefix);
//   k_key_collect the rows above the selected key, and the rows equal to it.
#include "tkdv_device.h"
#include "tkdv_extremes.h"
#include "tkdv_internal.h"

namespace tkdv {
namespace {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// Order-preserving map float -> uint32 (larger float, larger key).
__device__ __forceinline__ uint32_t max_key(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

template <int K>
__global__ void __launch_bounds__(kExtBlock) k_grid_max(ExtArgs a)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    constexpr int T = K / 8, Q = K / 4;
    constexpr int tab = T * Q * kWave * 16;  // FP32 table bytes
    {
        const uint4 *s0 = reinterpret_cast<const uint4 *>(a.phi_f32);
        uint4 *d = reinterpret_cast<uint4 *>(lds);
        for (int v = threadIdx.x; v < tab / 16; v += kExtBlock) d[v] = s0[v];
    }
    __syncthreads();
    const float4 *tb = reinterpret_cast<const float4 *>(lds);
    const int lane = threadIdx.x & 63, half = lane >> 5, pl = lane & 31;
    const unsigned long long n_tiles = (a.n + kTile - 1) / kTile;
    const unsigned long long waves = (unsigned long long)gridDim.x * (kExtBlock / kWave);
    unsigned long long n_exc = 0;
    for (unsigned long long tile = (unsigned long long)blockIdx.x * (kExtBlock / kWave) + (threadIdx.x >> 6);
         tile < n_tiles; tile += waves) {
        const unsigned long long row = tile * kTile + pl;
        const bool valid = row < a.n;
        const float4 *src = reinterpret_cast<const float4 *>(a.xhat + (valid ? row : 0ull) * a.stride + half * K);
        float x[K];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const float4 v = src[q];
            x[4 * q + 0] = v.x;
            x[4 * q + 1] = v.y;
            x[4 * q + 2] = v.z;
            x[4 * q + 3] = v.w;
        }
        float best = -INFINITY;
        int bj = 0;
        constexpr int kTileUnroll = T < 4 ? T : 2;  // grid tiles unrolled
#pragma unroll kTileUnroll
        for (int t = 0; t < T; ++t) {
            f32x16 acc = {};
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const float4 c = tb[(t * Q + q) * kWave + lane];
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(c.x, x[4 * q + 0], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(c.y, x[4 * q + 1], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(c.z, x[4 * q + 2], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(c.w, x[4 * q + 3], acc, 0, 0, 0);
            }
            // acc[v] of lane l: grid point 32 t + 8 (v/4) + 4 (l/32) + v%4 of row l%32;
            // v increases with the grid index within each half
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int j = 32 * t + 8 * (v >> 2) + 4 * half + (v & 3);
                if (acc[v] > best) {
                    best = acc[v];
                    bj = j;
                }
            }
        }
        // the other half of the row: larger value, or the lower index on a tie
        const float ob = __shfl_xor(best, 32, 64);
        const int oj = __shfl_xor(bj, 32, 64);
        if (ob > best || (ob == best && oj < bj)) {
            best = ob;
            bj = oj;
        }
        const float um = best * a.amp;
        const bool exc = valid && half == 0 && um > a.threshold;
        n_exc += __popcll(__ballot(exc));
        if (valid && half == 0) {
            a.keys[row] = max_key(um);
            if (a.umax) a.umax[row] = um;
            if (a.jmax) a.jmax[row] = bj;
        }
    }
    // n_exc is the same in every lane (sums of ballots)
    const unsigned long long tot = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(n_exc >> 32)) << 32) |
                                   __builtin_amdgcn_readfirstlane((uint32_t)n_exc);
    if (tot) atomicAdd(a.n_exceed, lane == 0 ? tot : 0ull);
}

// K = 64 and 128: the quarter-period form of the same grid maximum, on the
// grid xi_j = -pi + 2 pi j/N itself.  Representatives xi_rho = 2 pi rho/N,
// rho < K, from the FP32 statistics tables in LDS (16 rho per tile, outputs
// Ce, Co, Se, So: the cos/sin sums over even/odd modes); each gives u at
// xi (grid index 2K + rho), xi - pi (rho), -xi (2K - rho) and pi - xi
// (4K - rho), rho = 0 only the first two; +-pi/2 (3K and K) come from direct
// sums.  A quarter of the dense form's products.  A wave takes 16 rows at a
// time: lane l holds coordinates [K/4 (l/16), K/4 (l/16 + 1)) of both blocks
// of row l % 16 (the B operand of the 16x16x4 products, mode index on l/16).
template <int K>
struct ExtQ {
    static constexpr int CPL = K / 4, TILES = K / 16, QG = K / 32;
    static constexpr int TAB_BYTES = TILES * 4 * QG * kWave * 16;
    static constexpr int BLOCK = 512;
};

template <int K>
__global__ void __launch_bounds__(ExtQ<K>::BLOCK) k_grid_max_q(ExtArgs a)
{
    constexpr int CPL = ExtQ<K>::CPL, QG = ExtQ<K>::QG, B = ExtQ<K>::BLOCK;
    extern __shared__ __attribute__((aligned(16))) char lds[];
    {
        const uint4 *s0 = reinterpret_cast<const uint4 *>(a.phi_f32);
        uint4 *d = reinterpret_cast<uint4 *>(lds);
        for (int v = threadIdx.x; v < ExtQ<K>::TAB_BYTES / 16; v += B) d[v] = s0[v];
    }
    __syncthreads();
    const float4 *tab = reinterpret_cast<const float4 *>(lds);
    const int lane = threadIdx.x & 63, g = lane >> 4, pl = lane & 15;
    const unsigned long long n_chunks = (a.n + 15) / 16;
    const unsigned long long waves = (unsigned long long)gridDim.x * (B / kWave);
    unsigned long long n_exc = 0;
    for (unsigned long long ch = (unsigned long long)blockIdx.x * (B / kWave) + (threadIdx.x >> 6); ch < n_chunks;
         ch += waves) {
        const unsigned long long row = ch * 16 + pl;
        const bool valid = row < a.n;
        const float *src = a.xhat + (valid ? row : 0ull) * a.stride + CPL * g;
        float c[CPL], s[CPL];
#pragma unroll
        for (int q = 0; q < CPL / 4; ++q) {
            const float4 vc = reinterpret_cast<const float4 *>(src)[q];
            const float4 vs = reinterpret_cast<const float4 *>(src + K)[q];
            c[4 * q + 0] = vc.x;
            c[4 * q + 1] = vc.y;
            c[4 * q + 2] = vc.z;
            c[4 * q + 3] = vc.w;
            s[4 * q + 0] = vs.x;
            s[4 * q + 1] = vs.y;
            s[4 * q + 2] = vs.z;
            s[4 * q + 3] = vs.w;
        }
        float best = -INFINITY;
        int bj = 0x7fffffff;
        auto take = [&](float u, int j) {
            if (u > best || (u == best && j < bj)) {
                best = u;
                bj = j;
            }
        };
#pragma unroll 1
        for (int tau = 0; tau < ExtQ<K>::TILES; ++tau) {
            f32x4 acc[4] = {f32x4{}, f32x4{}, f32x4{}, f32x4{}};
#pragma unroll
            for (int q4 = 0; q4 < QG; ++q4)
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    // out o: 0 Ce, 1 Co, 2 Se, 3 So; mode K/4 g + 2 idx + 2 (even) or + 1 (odd)
                    const float4 av = tab[((tau * 4 + o) * QG + q4) * kWave + lane];
                    const float *v = (o < 2) ? c : s;
                    const int par = (o == 0 || o == 2) ? 1 : 0;
                    acc[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, v[2 * (4 * q4 + 0) + par], acc[o], 0, 0, 0);
                    acc[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, v[2 * (4 * q4 + 1) + par], acc[o], 0, 0, 0);
                    acc[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, v[2 * (4 * q4 + 2) + par], acc[o], 0, 0, 0);
                    acc[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, v[2 * (4 * q4 + 3) + par], acc[o], 0, 0, 0);
                }
#pragma unroll
            for (int v = 0; v < 4; ++v) {  // acc[o][v] of lane l: representative rho = 16 tau + 4 (l/16) + v
                const int rho = 16 * tau + 4 * g + v;
                const float pe = acc[0][v] + acc[1][v], me = acc[0][v] - acc[1][v];
                const float ps = acc[2][v] + acc[3][v], ms = acc[2][v] - acc[3][v];
                take(pe + ps, 2 * K + rho);  // xi
                take(me + ms, rho);          // xi - pi
                if (rho != 0) {
                    take(pe - ps, 2 * K - rho);  // -xi
                    take(me - ms, 4 * K - rho);  // pi - xi
                }
            }
        }
        // xi = +-pi/2: mode K g/4 + j + 1 is j + 1 modulo 4
        float Av = 0.0f, Bv = 0.0f;
#pragma unroll
        for (int j = 0; j < CPL; j += 4) {
            Av += c[j + 3] - c[j + 1];
            Bv += s[j] - s[j + 2];
        }
        Av += __shfl_xor(Av, 16, 64);
        Av += __shfl_xor(Av, 32, 64);
        Bv += __shfl_xor(Bv, 16, 64);
        Bv += __shfl_xor(Bv, 32, 64);
        if (g == 0) {
            take(Av + Bv, 3 * K);  // pi/2
            take(Av - Bv, K);      // -pi/2
        }
        // the row's grid values are split over lanes l, l ^ 16, l ^ 32, l ^ 48
#pragma unroll
        for (int m = 16; m <= 32; m <<= 1) {
            const float ob = __shfl_xor(best, m, 64);
            const int oj = __shfl_xor(bj, m, 64);
            take(ob, oj);
        }
        if (bj == 0x7fffffff) bj = 0;  // no value compared (a row of NaN)
        const float um = best * a.amp;
        const bool exc = valid && g == 0 && um > a.threshold;
        n_exc += __popcll(__ballot(exc));
        if (valid && g == 0) {
            a.keys[row] = max_key(um);
            if (a.umax) a.umax[row] = um;
            if (a.jmax) a.jmax[row] = bj;
        }
    }
    if (lane == 0 && n_exc) atomicAdd(a.n_exceed, n_exc);
}

__global__ void __launch_bounds__(256) k_key_hist(const uint32_t *keys, unsigned long long n, uint32_t prefix,
                                                 int shift, unsigned long long *hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    for (unsigned long long i = (unsigned long long)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * 256) {
        const uint32_t k = keys[i];
        const bool match = shift == 24 || (k >> (shift + 8)) == prefix;
        if (match) atomicAdd(&h[(k >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

__global__ void __launch_bounds__(256) k_key_collect(const uint32_t *keys, unsigned long long n, uint32_t kth,
                                                    unsigned long long *above, unsigned long long cap_above,
                                                    unsigned long long *equal, unsigned long long cap_equal,
                                                    unsigned long long *counts)
{
    for (unsigned long long i = (unsigned long long)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * 256) {
        const uint32_t k = keys[i];
        if (k > kth) {
            const unsigned long long pos = atomicAdd(&counts[0], 1ull);
            if (pos < cap_above) above[pos] = i;
        } else if (k == kth) {
            const unsigned long long pos = atomicAdd(&counts[1], 1ull);
            if (pos < cap_equal) equal[pos] = i;
        }
    }
}

__global__ void __launch_bounds__(256) k_ext_gather(const unsigned long long *rows, int n, const uint32_t *keys,
                                                   const int *jmax, uint32_t *okeys, int *ojmax)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const unsigned long long r = rows[i];
        okeys[i] = keys[r];
        ojmax[i] = jmax[r];
    }
}

}  // namespace

hipError_t launch_ext_gather(const unsigned long long *rows, int n, const uint32_t *keys, const int *jmax,
                             uint32_t *okeys, int *ojmax, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ext_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rows, n, keys, jmax, okeys,
                       ojmax);
    return hipGetLastError();
}

int ext_lds_bytes(int K) { return K >= 64 ? (K / 16) * 4 * (K / 32) * kWave * 16 : (K / 8) * (K / 4) * kWave * 16; }

template <int K>
hipError_t launch_grid_max_q(const ExtArgs &a, int n_cu, hipStream_t st)
{
    constexpr int lds = ExtQ<K>::TAB_BYTES, B = ExtQ<K>::BLOCK;
    auto kern = k_grid_max_q<K>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, B, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    const unsigned long long chunks = (a.n + 15) / 16;
    unsigned long long grid = (unsigned long long)per_cu * n_cu;
    const unsigned long long want = (chunks + B / kWave - 1) / (B / kWave);
    if (want < grid) grid = want;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(B), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_grid_max(int K, const ExtArgs &a, int n_cu, hipStream_t st)
{
    if (K == 64) return launch_grid_max_q<64>(a, n_cu, st);
    if (K == 128) return launch_grid_max_q<128>(a, n_cu, st);
    const int lds = ext_lds_bytes(K);
    const unsigned long long tiles = (a.n + kTile - 1) / kTile;
    unsigned long long grid = (unsigned long long)n_cu * 4;
    const unsigned long long want = (tiles + kExtBlock / kWave - 1) / (kExtBlock / kWave);
    if (want < grid) grid = want;
    if (grid < 1) grid = 1;
#define TKDV_EXT(KK)                                                                                     \
    case KK: {                                                                                           \
        hipError_t e = hipFuncSetAttribute((const void *)k_grid_max<KK>,                                 \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);             \
        if (e != hipSuccess) return e;                                                                   \
        hipLaunchKernelGGL(k_grid_max<KK>, dim3((unsigned)grid), dim3(kExtBlock), lds, st, a);           \
        break;                                                                                           \
    }
    switch (K) {
        TKDV_EXT(8)
        TKDV_EXT(16)
        TKDV_EXT(32)
    default: return hipErrorInvalidValue;
    }
#undef TKDV_EXT
    return hipGetLastError();
}

hipError_t launch_key_hist(const uint32_t *keys, unsigned long long n, uint32_t prefix, int shift,
                           unsigned long long *hist, int n_cu, hipStream_t st)
{
    unsigned long long g = (n + 255) / 256;
    if (g > (unsigned long long)n_cu * 8) g = (unsigned long long)n_cu * 8;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_key_hist, dim3((unsigned)g), dim3(256), 0, st, keys, n, prefix, shift, hist);
    return hipGetLastError();
}

hipError_t launch_key_collect(const uint32_t *keys, unsigned long long n, uint32_t kth, unsigned long long *above,
                              unsigned long long cap_above, unsigned long long *equal, unsigned long long cap_equal,
                              unsigned long long *counts, int n_cu, hipStream_t st)
{
    unsigned long long g = (n + 255) / 256;
    if (g > (unsigned long long)n_cu * 8) g = (unsigned long long)n_cu * 8;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_key_collect, dim3((unsigned)g), dim3(256), 0, st, keys, n, kth, above, cap_above, equal,
                       cap_equal, counts);
    return hipGetLastError();
}

}  // namespace tkdv
