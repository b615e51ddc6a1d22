// Sampling-importance resampling with the paper's proposals: launchers
// shared between tkdv_sir.hip and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tkdv_internal.h"

namespace tkdv {

constexpr int kSirChunk = 4096;   // tiles per block of the first scan level
constexpr int kSirPart = 8;       // FP64 partials per wave

struct SirArgs {
    const DevPoint *pt;           // the point (device)
    const void *phi_hi, *phi_lo;  // synthesis tables of the requested arithmetic
    unsigned long long n, n_tiles;
    float *w;                     // [n] weights f/(M g)
    double *tile_sum;             // [n_tiles] sum of the tile's weights
    double *wave_part;            // [waves][kSirPart]: sum w^2, max w, sum w S1..S4 (unscaled), # w > 1
    double *tile_off;             // [n_tiles] cumulative weight before the tile
    double *chunk_sum, *chunk_off;
    unsigned long long n_chunks;
    double W;                     // total weight (from the scan)
    double scale, u0;             // m/W and the systematic offset
    unsigned long long m;
    unsigned long long *index;    // [m] resampled proposal indices
    float *xhat;                  // [m][2K] rows or nullptr
};

int sir_block(int K);            // threads per workgroup of the weights kernel
int sir_waves(int K, int n_cu);  // waves of the weights kernel (one FP64 partial row each)
hipError_t launch_sir_weights(int K, int prec, int proposal, const SirArgs &a, int n_cu, hipStream_t st);
hipError_t launch_sir_scan(const SirArgs &a, hipStream_t st);
hipError_t launch_sir_resample(int K, int proposal, const SirArgs &a, int n_cu, hipStream_t st);

}  // namespace tkdv
