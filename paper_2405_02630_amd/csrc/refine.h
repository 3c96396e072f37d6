// FP64 refinement of large Gram entries (refine.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qsvm {

struct SweepArgs;

// Automatic threshold for n qubits: tiles whose largest computed entry
// exceeds it are recomputed in FP64.  The FP32 sweep's error at K = 1
// (self-overlaps, the largest amplitude) was measured at up to 3e-6 (64
// qubits), 8e-6 (400), 1.3e-5 (784) and 2.5e-5 (2000) over image, uniform
// and mixture features and reps 1..4, inside err(n) = 4e-6 + 2e-8 n.  The
// error of the amplitude is absolute (the environment stays O(1) after
// renormalisation), so an entry K carries |dK| <~ sqrt(K) err(n); entries
// left in FP32 stay within kRefineBudget (half the 1e-5 bar) when
// K <= (kRefineBudget / err(n))^2.  At or above 1 (n <= 50) nothing needs
// refining and the scan is skipped.
constexpr double kRefineBudget = 5e-6;
__host__ __device__ inline double auto_refine_threshold(int32_t n) {
  const double err = 4e-6 + 2e-8 * double(n);
  const double t = kRefineBudget / err;
  return t * t;
}

// After a sweep launch over the tiles of `a` (at most kMaxGridBlocks tiles):
// clear *count, list the tiles above `thresh` (list holds launch_tiles(a)
// entries) and recompute their pairs in FP64 with a grid of at most
// `resident_blocks` blocks.  reps 1..6.
hipError_t launch_refine(const SweepArgs& a, int32_t reps, double thresh, uint32_t* list, uint32_t* count,
                         int64_t resident_blocks, hipStream_t stream);
// FP64 entries of the pairs of a device-resident list (int32 (i, j) pairs,
// *count of them, clamped to [0, max_pairs]; invalid entries skipped) of the
// symmetric Gram described by `a`, with a grid of at most resident_blocks.
hipError_t launch_pairs_fp64(const SweepArgs& a, int32_t reps, const int32_t* pairs, const int32_t* count,
                             int64_t max_pairs, int64_t resident_blocks, hipStream_t stream);
// Blocks of the refinement kernel for `reps` resident on the current device.
hipError_t refine_resident_blocks(int32_t reps, int64_t* out);

}  // namespace qsvm
