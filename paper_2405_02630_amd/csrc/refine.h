// FP64 refinement of large Gram entries (refine.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qsvm {

struct SweepArgs;

// Default threshold: tiles whose largest computed entry exceeds it are
// recomputed in FP64.  Below it the FP32 sweep's relative error (< 1e-3 up
// to the largest supported qubit count, ~1.5e-5 at 784 qubits) keeps every
// entry within 1e-6 of exact.
constexpr double kDefaultRefineAbove = 1e-3;

// After a sweep launch over the tiles of `a` (at most kMaxGridBlocks tiles):
// clear *count, list the tiles above `thresh` (list holds launch_tiles(a)
// entries) and recompute their pairs in FP64 with a grid of at most
// `resident_blocks` blocks.  reps 1..4.
hipError_t launch_refine(const SweepArgs& a, int32_t reps, double thresh, uint32_t* list, uint32_t* count,
                         int64_t resident_blocks, hipStream_t stream);
// Blocks of the refinement kernel for `reps` resident on the current device.
hipError_t refine_resident_blocks(int32_t reps, int64_t* out);

}  // namespace qsvm
