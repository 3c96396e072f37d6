// Internal declarations shared by the C-ABI layer (api.cpp) and the HIP
// kernels.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qsvm {

// Bytes of section D (dense tensors) for N points.
inline int64_t dense_bytes(int64_t N, int32_t n, int32_t reps) {
  const int64_t chi = int64_t(1) << reps;
  return int64_t(n) * N * chi * chi * 8;
}

hipError_t launch_encode(const double* X, int64_t N, int32_t n, int32_t reps, void* mps,
                         hipStream_t stream);
struct SweepArgs;
constexpr int kButterflyVariants = 8;  // per reps, see launch_sweep_butterfly_args
hipError_t launch_sweep_butterfly_args(const SweepArgs& a, int32_t reps, int32_t variant, hipStream_t stream);
// Autotuned variant table (autotune.cpp).
int32_t tuned_variant(int32_t reps, int32_t n);
void set_tuned_variant(int32_t reps, int32_t n, int32_t variant);
hipError_t autotune_run(int32_t reps, int32_t n, int64_t N, hipStream_t stream, int32_t* best, float* ms_out);
hipError_t launch_sweep_dense_args(const SweepArgs& a, int32_t reps, hipStream_t stream);

}  // namespace qsvm
