// Host-side launchers of the gfx950 kernels (defined in tkdv_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "tkdv_internal.h"

namespace tkdv {

hipError_t launch_decide(int K, int prec, int prop, const KernelArgs &a, const int *plist, int n_plist,
                         int n_cu, unsigned long long total_tiles, hipStream_t st, int *grid_out);
hipError_t launch_decide_mix(int K, int prec, const KernelArgs &a, const int *plist, int n_plist, int n_cu,
                             unsigned long long total_tiles, hipStream_t st, int *grid_out);
// largest number of decide workgroups (paper's proposal) resident per compute unit
int decide_max_blocks_per_cu(int K, int prec);
// tile variants of the paper's-proposal decision kernel (variant 0: launch_decide)
hipError_t launch_decide_variant(int K, int prec, int prop, int variant, const KernelArgs &a, const int *plist,
                                 int n_plist, int n_cu, unsigned long long tiles, hipStream_t st, int *grid_out);
int decide_variant_block(int K, int variant);
int decide_variant_max_blocks_per_cu(int K, int prec, int variant);
hipError_t launch_fixup(const KernelArgs &a, int n_cu, hipStream_t st);
hipError_t launch_fixup_mix(int K, const KernelArgs &a, int n_cu, hipStream_t st);
hipError_t launch_segments(const KernelArgs &a, unsigned long long total_segs, unsigned long long *seg_cnt,
                           unsigned long long *seg_base, PointResult *res, int n_cu, hipStream_t st);
hipError_t launch_materialize(int K, int prop, const KernelArgs &a, const int *plist, int n_plist,
                              unsigned long long total_segs, const unsigned long long *seg_cnt,
                              const unsigned long long *seg_base, SegStats *seg_stats, PointResult *res,
                              float *out_xhat, unsigned long long *out_index, int n_cu, hipStream_t st);
hipError_t launch_finalize(const KernelArgs &a, const unsigned long long *seg_cnt,
                           const unsigned long long *seg_base, const SegStats *seg_stats, PointResult *res,
                           hipStream_t st);
// the standalone synthesis (tkdv_synth.hip); ev_start (optional) is recorded
// on st immediately before the kernel launch
hipError_t launch_synth(int K, int prec, const float *xhat, unsigned long long n, float *s3, const void *phi_hi,
                        const void *phi_lo, int n_cu, hipStream_t st, hipEvent_t ev_start, int *grid_out,
                        int *block_out);
// the same at K = 128 in the quarter-period form (tkdv_quarter.hip)
hipError_t launch_synth_quarter(int K, int prec, const float *xhat, unsigned long long n, float *s3,
                                const void *phi_hi, const void *phi_lo, int n_cu, hipStream_t st,
                                hipEvent_t ev_start, int *grid_out, int *block_out);
// Quarter-period form (tkdv_quarter.hip): the decision kernel at K = 128 and,
// as a tile variant, at K = 64; workgroup size, occupancy, the bytes of one
// table (FP32, or one BF16 table of hi/lo); the ordered output with
// statistics at K = 128
hipError_t launch_decide128(int prec, int prop, const KernelArgs &a, const int *plist, int n_plist, int n_cu,
                            unsigned long long total_tiles, hipStream_t st, int *grid_out);
hipError_t launch_decide_quarter64(int prec, int prop, const KernelArgs &a, const int *plist, int n_plist, int n_cu,
                                   unsigned long long total_tiles, hipStream_t st, int *grid_out);
int decide128_max_blocks_per_cu(int prec);
int decide_quarter64_max_blocks_per_cu(int prec);
// K = 128 tile variants (BF16x3, the paper's proposal); variant 0 is launch_decide128's
int decide128_n_variants();
int decide128_variant_block(int variant);
hipError_t launch_decide128_variant(int variant, const KernelArgs &a, const int *plist, int n_plist, int n_cu,
                                    unsigned long long total_tiles, hipStream_t st, int *grid_out);
int decide128_variant_max_blocks_per_cu(int variant);
// tile variants of K under the given arithmetic (1: the default kernel only)
int decide_n_variants(int K, int prec);
size_t quarter_table_bytes(int K, int prec);
// The ordered output and statistics at K = 64 and 128 (quarter-period form on
// the statistics grid; a.phi_hi: the table of upload_quarter_stats).
hipError_t launch_materialize_quarter(int K, int prop, const KernelArgs &a, unsigned long long total_segs,
                                     const unsigned long long *seg_cnt, const unsigned long long *seg_base,
                                     SegStats *seg_stats, PointResult *res, float *out_xhat,
                                     unsigned long long *out_index, int n_cu, hipStream_t st);
hipError_t launch_window_advance(DevPoint *pts, const DevCounters *cnt, const PointResult *res, SweepState *sw,
                                 int n_points, SweepGlobal *G, const unsigned long long *defer_count, hipStream_t st);
hipError_t launch_fill_u32(void *p, unsigned long long n_words, uint32_t v, hipStream_t st);
hipError_t launch_bits_to_bytes(const uint32_t *bitmap, unsigned long long n, uint8_t *out, hipStream_t st);

}  // namespace tkdv
