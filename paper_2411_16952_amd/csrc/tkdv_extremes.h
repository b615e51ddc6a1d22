// Extreme wave fields among stored samples: launchers shared with the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tkdv {

constexpr int kExtBlock = 256;  // threads per workgroup of k_grid_max (K <= 32)

struct ExtArgs {
    const float *xhat;          // [n][stride] rows of x^ (first 2K entries used)
    unsigned long long n, stride;
    const void *phi_f32;        // FP32 synthesis tables of K (K = 64, 128: quarter-period statistics tables)
    float amp;                  // sqrt(2 E0/pi)
    float threshold;            // rows with max u above it are counted
    uint32_t *keys;             // [n] order-preserving keys of the maxima
    float *umax;                // [n] or nullptr
    int *jmax;                  // [n] or nullptr
    unsigned long long *n_exceed;
};

int ext_lds_bytes(int K);
hipError_t launch_grid_max(int K, const ExtArgs &a, int n_cu, hipStream_t st);
hipError_t launch_key_hist(const uint32_t *keys, unsigned long long n, uint32_t prefix, int shift,
                           unsigned long long *hist, int n_cu, hipStream_t st);
hipError_t launch_key_collect(const uint32_t *keys, unsigned long long n, uint32_t kth, unsigned long long *above,
                              unsigned long long cap_above, unsigned long long *equal, unsigned long long cap_equal,
                              unsigned long long *counts, int n_cu, hipStream_t st);

hipError_t launch_ext_gather(const unsigned long long *rows, int n, const uint32_t *keys, const int *jmax,
                             uint32_t *okeys, int *ojmax, hipStream_t st);

}  // namespace tkdv
