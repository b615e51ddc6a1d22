// The fixed device scratch of tkdv_sample_noalloc (tkdv_scratch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace tkdv {

// Largest proposal range of one no-allocation call (n, or max_proposals in
// accepted-count mode), and the size of its FP64 re-decision list.
constexpr unsigned long long kScratchMaxProposals = 1ull << 26;
constexpr unsigned long long kScratchDeferCap = 1ull << 20;
// accept bitmap 8 MiB + re-decision list 8 MiB + 1 MiB for the counters,
// segment arrays and point records
constexpr size_t kScratchBytes = (kScratchMaxProposals / 32) * 4 + kScratchDeferCap * 8 + (1u << 20);

// Looks up the scratch array's address on `device` (made current for the
// call) once and keeps it; later calls return at once.
hipError_t scratch_init(int device);
// The kept address on `device`, or NULL before scratch_init.
void *scratch_ptr(int device);

}  // namespace tkdv
