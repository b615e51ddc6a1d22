// Quarter-period kernels of the TKdV rejection sampler at K = 64 and 128
// (N = 256, 512): the decision kernel, the ordered output with the
// statistics, and the standalone synthesis at K = 128.  The layout and the quarter-period synthesis are described
// in tkdv_quarter.h.
#include <hip/hip_runtime.h>

#include "tkdv_device.h"
#include "tkdv_kernels.h"
#include "tkdv_quarter.h"

namespace tkdv {

namespace {

// Work-queue claim as in the other decision kernels: every lane issues the
// atomic (lane 0 adds), lane 0's old value broadcast; ~0 when the target is met.
__device__ __forceinline__ unsigned long long claim128(const DevPoint &P, DevCounters *C, int lane)
{
    const bool open =
        P.target == ~0ull ||
        bcast0(__hip_atomic_load(&C->accepted, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < P.target;
    const unsigned long long old =
        atomicAdd(&C->next_tile, (open && lane == 0) ? (unsigned long long)kClaimTiles : 0ull);
    return open ? bcast0(old) : ~0ull;
}
__device__ __forceinline__ void add0(unsigned long long *ctr, unsigned long long v, int lane)
{
    if (bcast0(v) != 0ull) atomicAdd(ctr, lane == 0 ? v : 0ull);
}


// ---------------------------------------------------------------------------
// k_decide128: persistent; claims of 64 accept words (2048 proposals, 128
// tiles of 16) from per-point queues, as the other decision kernels.
// ---------------------------------------------------------------------------
// DBG: the verification entry's instantiation (per-proposal outputs written,
// workgroups of Quarter<K>::BLOCK); the sampling calls run the one without,
// which needs fewer registers.  BL: workgroup threads (decide_block(K), or a
// tile variant's).  |X| and t are finished before the synthesis: left for
// after it, the compiler keeps the sin block's 32 coordinates (K = 128) live
// through the products to sum their squares there, which leaves room for 2
// waves per SIMD instead of 3.
template <int K, int PREC, int PROP, bool DBG, int BL = decide_block(K)>
__global__ void __launch_bounds__(BL) k_decide128(KernelArgs a, const int *plist, int n_plist)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    constexpr int B = BL, CPL = K / 4;
    {
        const uint4 *s0 = reinterpret_cast<const uint4 *>(a.phi_hi);
        const uint4 *s1 = reinterpret_cast<const uint4 *>(a.phi_lo);
        uint4 *d = reinterpret_cast<uint4 *>(lds);
        constexpr int one = (PREC == PREC_FP32 ? Quarter<K>::F32_BYTES : Quarter<K>::BF16_BYTES) / 16;
        for (int v = threadIdx.x; v < one; v += B) d[v] = s0[v];
        if constexpr (PREC == PREC_BF16X3)
            for (int v = threadIdx.x; v < one; v += B) d[one + v] = s1[v];
    }
    __syncthreads();
    const char *lds_hi = lds;
    const char *lds_lo = lds + (PREC == PREC_FP32 ? 0 : Quarter<K>::BF16_BYTES);
    const int lane = threadIdx.x & 63, g = lane >> 4, pl = lane & 15;
    const int gwave = blockIdx.x * (B / kWave) + (threadIdx.x >> 6);
    int cursor = gwave % n_plist;
    int misses = 0;
    while (misses < n_plist) {
        const int p = __builtin_amdgcn_readfirstlane(plist[cursor]);
        const DevPoint &P = a.pts[p];
        DevCounters *C = a.cnt + p;
        const unsigned long long base = claim128(P, C, lane);
        if (base >= P.n_tiles) {
            cursor = (cursor + 1 == n_plist) ? 0 : cursor + 1;
            ++misses;
            continue;
        }
        misses = 0;
        unsigned long long n_acc = 0, n_def = 0;
        unsigned int n_viol = 0;
        float max_la = -INFINITY;
        uint32_t my_word = 0u;  // accept bits of word `lane` of this claim
        for (int c2 = 0; c2 < 2 * kClaimTiles; ++c2) {
            const unsigned long long word = base + (c2 >> 1);
            if (word >= P.n_tiles) break;
            const unsigned long long local = word * kTile + (c2 & 1) * kTile16 + pl;
            const bool valid = local < P.n;
            const uint64_t i = P.i0 + local;
            if (DBG && a.dbg_xhat) {  // verification: the projected point, generated once more
                float c[CPL], s[CPL], tt;
                uint32_t ww;
                gen_x128<K, PROP, true, true>(P, i, g, c, s, tt, ww);  // the decision's draw
                if (valid) {
                    float *row = a.dbg_xhat + local * (2 * K);
#pragma unroll
                    for (int j = 0; j < CPL; ++j) {
                        row[CPL * g + j] = c[j];
                        row[K + CPL * g + j] = s[j];
                    }
                }
            }
            const uint32_t c0 = (uint32_t)i, c1 = (uint32_t)(i >> 32);
            float r2 = 0.0f, a1 = 0.0f, a2 = 0.0f, s3l, t, inv;
            if constexpr (PREC == PREC_FP32) {
                float c[CPL], s[CPL];
                gen_block128<K, PROP>(P, c0, c1, g, 0, c, r2, a1, a2);
                gen_block128<K, PROP>(P, c0, c1, g, 1, s, r2, a1, a2);
                inv = finish_norm128<K>(g, r2, a1, a2, t);
                __builtin_amdgcn_sched_barrier(0);
                s3l = cube_sum_q128_f32<K>(c, s, lds_hi, lane);
            } else {
                // one block at a time: its coordinates die once split into operands
                constexpr int R = Quarter<K>::STEPS;
                bf16x8 bh[4][R], bl[4][R];
#pragma unroll
                for (int blk = 0; blk < 2; ++blk) {
                    float v[CPL];
                    gen_block128<K, PROP>(P, c0, c1, g, blk, v, r2, a1, a2);
#pragma unroll
                    for (int odd = 0; odd < 2; ++odd)
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            quarter_operand<CPL, PREC == PREC_BF16X3>(v, odd, r, bh[2 * blk + odd][r],
                                                                      bl[2 * blk + odd][r]);
                    // keep the next block's generation after this split (register pressure)
                    __builtin_amdgcn_sched_barrier(0);
                }
                inv = finish_norm128<K>(g, r2, a1, a2, t);
                __builtin_amdgcn_sched_barrier(0);
                s3l = cube_sum_q128_bf16<K, PREC, K == 128 ? 2 : 1>(bh, bl, lds_hi, lds_lo, lane);
            }
            const uint32_t w_acc = philox4x32_10(c0, c1, P.point_id, (uint32_t)(K / 2), P.key0, P.key1).x;
            const float s3 = sum4(s3l) * (inv * inv * inv);
            const float la = log_a_f32<PROP>(P, t, s3);
            const float U = __builtin_fmaf((float)w_acc, 2.3283064365386963e-10f, 1.1641532182693481e-10f);
            const float alin = __builtin_amdgcn_exp2f(la * 1.4426950408889634f);
            const float lo_edge = alin * P.e_lo, hi_edge = alin * P.e_hi;
            const bool mine = valid && g == 0;
            // above the bound by no more than the fast path's error (0 < log a <= tau):
            // the decision and the check of eq. (M_sup) are left to the FP64 pass
            const bool near_bound = la > 0.0f && la <= P.tau;
            const bool defer = mine && ((U >= lo_edge && U < hi_edge) || near_bound);
            const bool accept = mine && U < lo_edge && !near_bound;
            const unsigned long long bacc = __ballot(accept);
            const unsigned long long bdef = __ballot(defer);
            if (lane == (c2 >> 1)) my_word |= (uint32_t)(bacc & 0xffffull) << (16 * (c2 & 1));
            n_acc += __popcll(bacc);
            if (mine) {
                n_viol += (la > 0.0f && !defer) ? 1u : 0u;  // window proposals: k_fixup
                max_la = fmaxf(max_la, la);
                if (DBG && a.dbg_t) {
                    a.dbg_t[local] = t;
                    a.dbg_s3[local] = s3;
                    a.dbg_log_a[local] = la;
                    a.dbg_log_u[local] = log_u_word(w_acc);
                }
            }
            if (bdef) {
                const unsigned long long nd = __popcll(bdef);
                const unsigned long long slot = bcast0(atomicAdd(a.defer_count, lane == 0 ? nd : 0ull));
                if (defer) {
                    const unsigned long long pos = slot + __popcll(bdef & ((1ull << lane) - 1ull));
                    if (pos < a.defer_cap) a.defer_list[pos] = pack_defer(p, i);
                }
                n_def += nd;
            }
        }
        if (base + lane < P.n_tiles) a.bitmap[P.bm_off + base + lane] = my_word;
        const unsigned long long viol = wave_sum_u64_128(n_viol);
        max_la = wave_max_128(max_la);
        add0(&C->accepted, n_acc, lane);
        add0(&C->violations, viol, lane);
        add0(&C->deferred, n_def, lane);
        if (__builtin_amdgcn_readfirstlane(__float_as_uint(max_la)) != __float_as_uint(-INFINITY))
            atomicMax(&C->max_log_a_key, lane == 0 ? float_key(max_la) : 0u);
    }
}

// ---------------------------------------------------------------------------
// k_materialize_q: the ordered output and the statistics at K = 64 and 128.
// One workgroup per 65536-proposal segment, its W waves taking equal runs of
// its accept words in groups of 32; accepted proposals in chunks of 16 (the
// decision kernel's layout), regenerated with the decision kernel's
// arithmetic and written at their rank.  The grid values come from the
// quarter-period form on the statistics grid xi_j = -pi + 2 pi j/N itself:
// representatives xi_rho = 2 pi rho/N, rho < K (FP32 16x16x4 products, table
// in LDS, entries unscaled), each giving u at xi, -xi, pi - xi and xi - pi
// from Ce, Co, Se, So; rho = 0 has only the two points 0 and pi, and the
// points +-pi/2 (rho = K) come from direct sums: cos(k pi/2) and sin(k pi/2)
// are 0 or +-1.  Each wave queues its accepted offsets in LDS, in index order,
// and regenerates full chunks only (the last group flushes the rest): at an
// acceptance of 1e-3 a group of 32 words holds one accepted proposal.
// ---------------------------------------------------------------------------
template <int K>
struct MatQ {
    static constexpr int W = K == 128 ? 8 : 4;       // waves per workgroup
    static constexpr int WAVE_WORDS = kSegWords / W; // accept words per wave
    static constexpr int GROUP = 32;                 // words per group (lanes 0..31)
    static constexpr int QUEUE = GROUP * 32 + 16;    // one group's offsets + a partial chunk
    static constexpr int LIST_BYTES = W * QUEUE * 2;
    static constexpr int LDS = Quarter<K>::F32_BYTES + LIST_BYTES;
};

template <int K, int PROP>
__global__ void __launch_bounds__(MatQ<K>::W * kWave) k_materialize_q(KernelArgs a, unsigned long long total_segs,
                                                                      const unsigned long long *seg_cnt,
                                                                      const unsigned long long *seg_base,
                                                                      SegStats *seg_stats, PointResult *res,
                                                                      float *out_xhat, unsigned long long *out_index)
{
    constexpr int W = MatQ<K>::W, B = W * kWave, CPL = K / 4, QG = Quarter<K>::QG;
    constexpr int WW = MatQ<K>::WAVE_WORDS, GW = MatQ<K>::GROUP;
    extern __shared__ __attribute__((aligned(16))) char lds[];
    __shared__ unsigned int hist[kNBins];
    __shared__ unsigned long long wave_cnt[W];
    __shared__ double wave_S[W][4];
    __shared__ unsigned long long wave_ex[W][3];
    __shared__ unsigned long long wave_peak_idx[W];
    __shared__ unsigned int wave_peak_key[W];
    {
        const uint4 *s0 = reinterpret_cast<const uint4 *>(a.phi_hi);
        uint4 *d = reinterpret_cast<uint4 *>(lds);
        for (int v = threadIdx.x; v < Quarter<K>::F32_BYTES / 16; v += B) d[v] = s0[v];
    }
    const float4 *tab = reinterpret_cast<const float4 *>(lds);
    const int lane = threadIdx.x & 63, g = lane >> 4, pl = lane & 15, wv = threadIdx.x >> 6;
    uint16_t *mylist = reinterpret_cast<uint16_t *>(lds + Quarter<K>::F32_BYTES) + wv * MatQ<K>::QUEUE;
    if (a.d_total_segs) total_segs = *a.d_total_segs;
    __syncthreads();
    for (unsigned long long gs = blockIdx.x; gs < total_segs; gs += gridDim.x) {
        int lo = 0, hi = a.n_points - 1;
        while (lo < hi) {  // last point whose first segment is <= gs
            const int mid = (lo + hi + 1) >> 1;
            if (a.pts[mid].seg_off <= gs) lo = mid; else hi = mid - 1;
        }
        const int p = lo;
        const DevPoint &P = a.pts[p];
        const unsigned long long limit = P.target;  // ranks >= target are not part of the result
        if (P.K != K || P.proposal != PROP || seg_cnt[gs] == 0 || seg_base[gs] >= limit) continue;  // uniform
        for (int b = threadIdx.x; b < kNBins; b += B) hist[b] = 0u;
        const unsigned long long nt = a.cnt[p].next_tile;
        const unsigned long long nw = nt < P.n_tiles ? nt : P.n_tiles;
        const unsigned long long w_first = (gs - P.seg_off) * kSegWords + (unsigned long long)wv * WW;
        unsigned long long cw = 0;
        for (int k = lane; k < WW; k += kWave) {
            const unsigned long long w = w_first + k;
            if (w < nw) cw += __popc(a.bitmap[P.bm_off + w]);
        }
        cw = wave_sum_u64_128(cw);
        if (lane == 0) wave_cnt[wv] = cw;
        __syncthreads();
        unsigned long long rank = seg_base[gs];
        for (int w = 0; w < wv; ++w) rank += wave_cnt[w];
        double S1 = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0;
        unsigned long long n_ex = 0, n_ex4 = 0, n_max4 = 0, peak_idx = ~0ull;
        unsigned int peak_key = 0u;
        int queued = 0;  // offsets (proposals from the wave's first word) waiting in mylist
        for (int grp = 0; grp < WW / GW; ++grp) {
            const unsigned long long w = w_first + (unsigned long long)grp * GW + lane;
            const uint32_t word = (lane < GW && w < nw) ? a.bitmap[P.bm_off + w] : 0u;
            const int cntw = __popc(word);
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
                mylist[pos++] = (uint16_t)((grp * GW + lane) * 32 + bit);
            }
            queued += total;
            const int upto = grp + 1 == WW / GW ? queued : queued & ~(kTile16 - 1);
            if (upto == 0) continue;
            // the list is written and read by lanes of this wave only
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (int c0 = 0; c0 < upto; c0 += kTile16) {
                const bool in_chunk = c0 + pl < upto;
                const int off = in_chunk ? (int)mylist[c0 + pl] : 0;
                const unsigned long long local = w_first * kTile + (unsigned long long)off;
                const uint64_t i = P.i0 + local;
                const unsigned long long r = rank + c0 + pl;
                const bool valid = in_chunk && r < limit;
                float c[CPL], s[CPL], t;
                uint32_t w_acc;
                gen_x128<K, PROP, true>(P, i, g, c, s, t, w_acc);
                if (valid && r < P.capacity) {
                    if (out_xhat) {
                        float *row = out_xhat + (P.out_off + r) * P.row_stride;
#pragma unroll
                        for (int j = 0; j < CPL; ++j) {
                            row[CPL * g + j] = c[j];
                            row[K + CPL * g + j] = s[j];
                        }
                    }
                    if (out_index && g == 0) out_index[P.out_off + r] = i;
                }
                if (valid && g == 0 && r + 1 == limit) a.cnt[p].last_index = i;
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
#pragma unroll 1
                for (int tau = 0; tau < Quarter<K>::TILES; ++tau) {
                    f32x4 acc[4] = {f32x4{}, f32x4{}, f32x4{}, f32x4{}};
#pragma unroll
                    for (int q4 = 0; q4 < QG; ++q4)
#pragma unroll
                        for (int o = 0; o < 4; ++o) {
                            // out o: 0 Ce, 1 Co, 2 Se, 3 So; coordinate 2 idx + 1 (even mode) or 2 idx (odd)
                            const float4 av = tab[((tau * 4 + o) * QG + q4) * 64 + lane];
                            const float *v = (o < 2) ? c : s;
                            const int par = (o == 0 || o == 2) ? 1 : 0;
                            acc[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, v[2 * (4 * q4 + 0) + par], acc[o], 0, 0, 0);
                            acc[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, v[2 * (4 * q4 + 1) + par], acc[o], 0, 0, 0);
                            acc[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, v[2 * (4 * q4 + 2) + par], acc[o], 0, 0, 0);
                            acc[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, v[2 * (4 * q4 + 3) + par], acc[o], 0, 0, 0);
                        }
                    if (valid) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) {  // representative rho = 16 tau + 4 g + v
                            const float pe = acc[0][v] + acc[1][v], me = acc[0][v] - acc[1][v];
                            const float ps = acc[2][v] + acc[3][v], ms = acc[2][v] - acc[3][v];
                            fold(pe + ps);  // xi
                            fold(me + ms);  // xi - pi
                            if (tau != 0 || v != 0 || g != 0) {  // rho = 0: xi = 0 and pi only
                                fold(pe - ps);  // -xi
                                fold(me - ms);  // pi - xi
                            }
                        }
                    }
                }
                // xi = +-pi/2: A = sum_k a_k cos(k pi/2), B = sum_k b_k sin(k pi/2); mode
                // K g/4 + j + 1 is j + 1 modulo 4
                float Av = 0.0f, Bv = 0.0f;
#pragma unroll
                for (int j = 0; j < CPL; j += 4) {
                    Av += c[j + 3] - c[j + 1];
                    Bv += s[j] - s[j + 2];
                }
                Av = sum4(Av);
                Bv = sum4(Bv);
                if (valid && g == 0) {
                    fold(Av + Bv);
                    fold(Av - Bv);
                }
                // the proposal's grid values are split over lanes l, l ^ 16, l ^ 32, l ^ 48
                umax = fmaxf(umax, __shfl_xor(umax, 16, 64));
                umax = fmaxf(umax, __shfl_xor(umax, 32, 64));
                // u(0) = sqrt(2 E0/pi) sum_k x^_k; bin of u(0)/u_max = sum_k x^_k / sqrt(K)
                double s0 = 0.0;
#pragma unroll
                for (int j = 0; j < CPL; ++j) s0 += (double)c[j];
                s0 += __shfl_xor(s0, 16, 64);
                s0 += __shfl_xor(s0, 32, 64);
                if (valid && g == 0) {
                    n_max4 += umax > kFourSigmaT ? 1ull : 0ull;
                    peak_merge(peak_key, peak_idx, float_key(umax), i);
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
        S1 = wave_sum_f64_128(S1);
        S2 = wave_sum_f64_128(S2);
        S3 = wave_sum_f64_128(S3);
        S4 = wave_sum_f64_128(S4);
        n_ex = wave_sum_u64_128(n_ex);
        n_ex4 = wave_sum_u64_128(n_ex4);
        n_max4 = wave_sum_u64_128(n_max4);
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
            for (int w = 0; w < W; ++w) {
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
        for (int b = threadIdx.x; b < kNBins; b += B)
            if (hist[b]) atomicAdd(&res[p].hist[b], (unsigned long long)hist[b]);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// k_synth_q: the standalone synthesis (rows of x^ in HBM -> S3 = sum of the
// cubes of the grid values of each row) at K = 128, in the quarter-period form
// on the grid offset by half a step, whose trapezoid sum of u~^3 equals that on
// xi_j = -pi + 2 pi j/N (both are exact for N >= 3K + 1), with the decision
// kernel's tables and arithmetic.
// ---------------------------------------------------------------------------  Sixteen
// rows per wave: lane l holds coordinates K/4 (l/16) .. K/4 (l/16) + K/4 - 1 of
// both blocks of row l % 16 (the column operand of the 16x16 products); the
// BF16 paths split each block into operands as it arrives.  Workgroups of
// Quarter<K>::BLOCK threads share the tables (128 KB for FP32 and BF16x3).
template <int K, int PREC>
__global__ void __launch_bounds__(Quarter<K>::BLOCK) k_synth_q(const float *__restrict__ xhat, unsigned long long n,
                                                               float *__restrict__ s3_out, const void *phi_hi,
                                                               const void *phi_lo)
{
    constexpr int B = Quarter<K>::BLOCK, CPL = K / 4, R = Quarter<K>::STEPS;
    constexpr int one = (PREC == PREC_FP32 ? Quarter<K>::F32_BYTES : Quarter<K>::BF16_BYTES) / 16;
    extern __shared__ __attribute__((aligned(16))) char lds[];
    {
        const uint4 *s0 = reinterpret_cast<const uint4 *>(phi_hi);
        const uint4 *s1 = reinterpret_cast<const uint4 *>(phi_lo);
        uint4 *d = reinterpret_cast<uint4 *>(lds);
        for (int v = threadIdx.x; v < one; v += B) d[v] = s0[v];
        if constexpr (PREC == PREC_BF16X3)
            for (int v = threadIdx.x; v < one; v += B) d[one + v] = s1[v];
    }
    __syncthreads();
    const char *lds_hi = lds, *lds_lo = lds + (PREC == PREC_BF16X3 ? one * 16 : 0);
    const int lane = threadIdx.x & 63, g = lane >> 4, pl = lane & 15;
    const unsigned long long n_chunks = (n + 15) / 16;
    const unsigned long long waves = (unsigned long long)gridDim.x * (B / kWave);
    for (unsigned long long ch = (unsigned long long)blockIdx.x * (B / kWave) + (threadIdx.x >> 6); ch < n_chunks;
         ch += waves) {
        const unsigned long long row = ch * 16 + pl;
        const bool valid = row < n;
        const float *src = xhat + (valid ? row : 0ull) * (2 * K) + CPL * g;
        auto load = [&](int blk, float (&v)[CPL]) {
            const float4 *p = reinterpret_cast<const float4 *>(src + blk * K);
#pragma unroll
            for (int q = 0; q < CPL / 4; ++q) {
                const float4 w = p[q];
                v[4 * q + 0] = w.x;
                v[4 * q + 1] = w.y;
                v[4 * q + 2] = w.z;
                v[4 * q + 3] = w.w;
            }
        };
        float s3l;
        if constexpr (PREC == PREC_FP32) {
            float c[CPL], s[CPL];
            load(0, c);
            load(1, s);
            s3l = cube_sum_q128_f32<K>(c, s, lds_hi, lane);
        } else {
            bf16x8 bh[4][R], bl[4][R];
#pragma unroll
            for (int blk = 0; blk < 2; ++blk) {
                float v[CPL];
                load(blk, v);
#pragma unroll
                for (int odd = 0; odd < 2; ++odd)
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        quarter_operand<CPL, PREC == PREC_BF16X3>(v, odd, r, bh[2 * blk + odd][r], bl[2 * blk + odd][r]);
            }
            s3l = cube_sum_q128_bf16<K, PREC>(bh, bl, lds_hi, lds_lo, lane);
        }
        const float s3 = sum4(s3l);
        if (valid && g == 0) s3_out[row] = s3;
    }
}

template <int K, int PREC>
hipError_t launch_synth_q_t(const float *xhat, unsigned long long n, float *s3, const void *phi_hi,
                            const void *phi_lo, int n_cu, hipStream_t st, hipEvent_t ev_start, int *grid_out,
                            int *block_out)
{
    constexpr int B = Quarter<K>::BLOCK;
    constexpr int lds = PREC == PREC_FP32 ? Quarter<K>::F32_BYTES
                                          : (PREC == PREC_BF16X3 ? 2 : 1) * Quarter<K>::BF16_BYTES;
    auto kern = k_synth_q<K, PREC>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, B, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    const unsigned long long chunks = (n + 15) / 16;
    unsigned long long grid = (unsigned long long)per_cu * n_cu;
    const unsigned long long want = (chunks + B / kWave - 1) / (B / kWave);
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

template <int K, int PROP>
hipError_t launch_materialize_q_t(const KernelArgs &a, unsigned long long total_segs,
                                  const unsigned long long *seg_cnt, const unsigned long long *seg_base,
                                  SegStats *seg_stats, PointResult *res, float *out_xhat,
                                  unsigned long long *out_index, int n_cu, hipStream_t st)
{
    constexpr int lds = MatQ<K>::LDS, B = MatQ<K>::W * kWave;
    auto kern = k_materialize_q<K, PROP>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, B, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    unsigned long long g = (unsigned long long)per_cu * n_cu;
    if (total_segs < g) g = total_segs;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)g), dim3(B), lds, st, a, total_segs, seg_cnt, seg_base, seg_stats, res,
                       out_xhat, out_index);
    return hipGetLastError();
}

template <int K, int PREC, int PROP, int BL = decide_block(K)>
hipError_t launch_decide128_t(const KernelArgs &a, const int *plist, int n_plist, int n_cu,
                              unsigned long long total_tiles, hipStream_t st, int *grid_out)
{
    constexpr int lds = Quarter<K>::lds(PREC), BD = Quarter<K>::BLOCK;
    const bool dbg = a.dbg_xhat != nullptr || a.dbg_t != nullptr;
    const int B = dbg ? BD : BL;
    auto kern = dbg ? k_decide128<K, PREC, PROP, true, BD> : k_decide128<K, PREC, PROP, false, BL>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, B, lds);
    if (e != hipSuccess) return e;
    if (a.blocks_per_cu > 0 && a.blocks_per_cu < per_cu) per_cu = a.blocks_per_cu;
    if (per_cu < 1) per_cu = 1;
    const unsigned long long per_block = (unsigned long long)(B / kWave) * kClaimTiles;
    unsigned long long want = (total_tiles + per_block - 1) / per_block;
    unsigned long long grid = (unsigned long long)per_cu * n_cu;
    if (want < grid) grid = want;
    if (grid < 1) grid = 1;
    if (grid_out) *grid_out = (int)grid;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(B), lds, st, a, plist, n_plist);
    return hipGetLastError();
}

template <int K, int PREC, int PROP, int BL = decide_block(K)>
int blocks_per_cu128_t()
{
    constexpr int lds = Quarter<K>::lds(PREC);
    auto kern = k_decide128<K, PREC, PROP, false, BL>;
    if (hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
        return 1;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, BL, lds) != hipSuccess) return 1;
    return per_cu < 1 ? 1 : per_cu;
}

// Tile variants at K = 128 (BF16x3, the paper's proposal): workgroups of 768
// threads (the default: 3 waves per SIMD, no register spills), 512 (2 waves
// per SIMD) and 1024 (4 waves per SIMD, some 13 registers spilled).
constexpr int kVariants128 = 3;
constexpr int kVariant128Block[kVariants128] = {decide_block(128), 512, 1024};

template <int K>
hipError_t launch_quarter_k(int prec, int prop, const KernelArgs &a, const int *plist, int n_plist, int n_cu,
                            unsigned long long total_tiles, hipStream_t st, int *grid_out)
{
    if (prec == PREC_FP32 && prop == PROP_UNIFORM)
        return launch_decide128_t<K, PREC_FP32, PROP_UNIFORM>(a, plist, n_plist, n_cu, total_tiles, st, grid_out);
    if (prec == PREC_FP32 && prop == PROP_SIGMA)
        return launch_decide128_t<K, PREC_FP32, PROP_SIGMA>(a, plist, n_plist, n_cu, total_tiles, st, grid_out);
    if (prec == PREC_BF16X3 && prop == PROP_UNIFORM)
        return launch_decide128_t<K, PREC_BF16X3, PROP_UNIFORM>(a, plist, n_plist, n_cu, total_tiles, st,
                                                                grid_out);
    if (prec == PREC_BF16X3 && prop == PROP_SIGMA)
        return launch_decide128_t<K, PREC_BF16X3, PROP_SIGMA>(a, plist, n_plist, n_cu, total_tiles, st,
                                                              grid_out);
    return hipErrorInvalidValue;
}

}  // namespace

size_t quarter_table_bytes(int K, int prec)
{
    if (K == 64) return prec == PREC_FP32 ? Quarter<64>::F32_BYTES : Quarter<64>::BF16_BYTES;
    return prec == PREC_FP32 ? Quarter<128>::F32_BYTES : Quarter<128>::BF16_BYTES;
}

hipError_t launch_decide128(int prec, int prop, const KernelArgs &a, const int *plist, int n_plist, int n_cu,
                            unsigned long long total_tiles, hipStream_t st, int *grid_out)
{
    return launch_quarter_k<128>(prec, prop, a, plist, n_plist, n_cu, total_tiles, st, grid_out);
}

hipError_t launch_decide_quarter64(int prec, int prop, const KernelArgs &a, const int *plist, int n_plist, int n_cu,
                                   unsigned long long total_tiles, hipStream_t st, int *grid_out)
{
    return launch_quarter_k<64>(prec, prop, a, plist, n_plist, n_cu, total_tiles, st, grid_out);
}

int decide128_n_variants() { return kVariants128; }
int decide128_variant_block(int variant)
{
    return variant > 0 && variant < kVariants128 ? kVariant128Block[variant] : decide_block(128);
}

hipError_t launch_decide128_variant(int variant, const KernelArgs &a, const int *plist, int n_plist, int n_cu,
                                    unsigned long long total_tiles, hipStream_t st, int *grid_out)
{
    if (variant == 1)
        return launch_decide128_t<128, PREC_BF16X3, PROP_SIGMA, kVariant128Block[1]>(a, plist, n_plist, n_cu,
                                                                                   total_tiles, st, grid_out);
    if (variant == 2)
        return launch_decide128_t<128, PREC_BF16X3, PROP_SIGMA, kVariant128Block[2]>(a, plist, n_plist, n_cu,
                                                                                   total_tiles, st, grid_out);
    return launch_decide128_t<128, PREC_BF16X3, PROP_SIGMA>(a, plist, n_plist, n_cu, total_tiles, st, grid_out);
}

int decide128_variant_max_blocks_per_cu(int variant)
{
    if (variant == 1) return blocks_per_cu128_t<128, PREC_BF16X3, PROP_SIGMA, kVariant128Block[1]>();
    if (variant == 2) return blocks_per_cu128_t<128, PREC_BF16X3, PROP_SIGMA, kVariant128Block[2]>();
    return blocks_per_cu128_t<128, PREC_BF16X3, PROP_SIGMA>();
}

int decide128_max_blocks_per_cu(int prec)
{
    return prec == PREC_FP32 ? blocks_per_cu128_t<128, PREC_FP32, PROP_SIGMA>()
                             : blocks_per_cu128_t<128, PREC_BF16X3, PROP_SIGMA>();
}

int decide_quarter64_max_blocks_per_cu(int prec)
{
    return prec == PREC_FP32 ? blocks_per_cu128_t<64, PREC_FP32, PROP_SIGMA>()
                             : blocks_per_cu128_t<64, PREC_BF16X3, PROP_SIGMA>();
}

hipError_t launch_materialize_quarter(int K, int prop, const KernelArgs &a, unsigned long long total_segs,
                                     const unsigned long long *seg_cnt, const unsigned long long *seg_base,
                                     SegStats *seg_stats, PointResult *res, float *out_xhat,
                                     unsigned long long *out_index, int n_cu, hipStream_t st)
{
#define TKDV_DISPATCH_MQ(KK, PP)                                                                            \
    if (K == KK && prop == PP)                                                                             \
        return launch_materialize_q_t<KK, PP>(a, total_segs, seg_cnt, seg_base, seg_stats, res, out_xhat, \
                                              out_index, n_cu, st);
    TKDV_DISPATCH_MQ(64, PROP_SIGMA)
    TKDV_DISPATCH_MQ(64, PROP_UNIFORM)
    TKDV_DISPATCH_MQ(128, PROP_SIGMA)
    TKDV_DISPATCH_MQ(128, PROP_UNIFORM)
#undef TKDV_DISPATCH_MQ
    return hipErrorInvalidValue;
}

hipError_t launch_synth_quarter(int K, int prec, const float *xhat, unsigned long long n, float *s3,
                                const void *phi_hi, const void *phi_lo, int n_cu, hipStream_t st,
                                hipEvent_t ev_start, int *grid_out, int *block_out)
{
    if (K != 128) return hipErrorInvalidValue;
    if (prec == PREC_FP32)
        return launch_synth_q_t<128, PREC_FP32>(xhat, n, s3, phi_hi, phi_lo, n_cu, st, ev_start, grid_out, block_out);
    if (prec == PREC_BF16)
        return launch_synth_q_t<128, PREC_BF16>(xhat, n, s3, phi_hi, phi_lo, n_cu, st, ev_start, grid_out, block_out);
    if (prec == PREC_BF16X3)
        return launch_synth_q_t<128, PREC_BF16X3>(xhat, n, s3, phi_hi, phi_lo, n_cu, st, ev_start, grid_out,
                                                  block_out);
    return hipErrorInvalidValue;
}

}  // namespace tkdv
