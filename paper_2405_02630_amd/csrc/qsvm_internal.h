// Internal declarations shared by the C-ABI layer (api.cpp) and the HIP
// kernels.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace qsvm {

// Bytes of the dense site tensors (the buffer of qsvm_encode_dense) for N points.
inline int64_t dense_bytes(int64_t N, int32_t n, int32_t reps) {
  const int64_t chi = int64_t(1) << reps;
  return int64_t(n) * N * chi * chi * 8;
}
// Bytes of the MPS buffer: Section G (generators), then Section L (their
// residuals), 16 B per site and point each.
inline int64_t mps_total_bytes(int64_t N, int32_t n, int32_t /*reps*/) { return int64_t(n) * N * 32; }

// Sections G and L into mps; the dense tensors into their own buffer.
hipError_t launch_encode(const double* X, int64_t N, int32_t n, int32_t reps, void* mps,
                         hipStream_t stream);
hipError_t launch_encode_dense(const double* X, int64_t N, int32_t n, int32_t reps, void* dense,
                               hipStream_t stream);
struct SweepArgs;
constexpr int kButterflyVariants = 4;  // per reps, see launch_sweep_butterfly_args
// Sites between power-of-two renormalisations of the FP32 environment: the
// default and the largest accepted interval.  Within one interval the
// largest entry can grow by at most 2^(2r-1) per site (each butterfly axis at
// most doubles it), 2^80 over 16 sites at r = 3, far from FP32 overflow; it
// underflows the FP32 normal range only if it shrinks by more than 2^-125
// within one interval, i.e. by a factor below 2^-15.6 per site on average
// over 8 sites.
constexpr int32_t kDefaultRenorm = 8;
constexpr int32_t kMaxRenorm = 16;
constexpr int32_t kMaxReps = 6;        // chi = 64
constexpr int32_t kMaxDenseReps = 4;   // dense site tensors (chi <= 16) are written up to here
hipError_t launch_sweep_butterfly_args(const SweepArgs& a, int32_t reps, int32_t variant, hipStream_t stream);
int32_t butterfly_variant_pi(int32_t reps, int32_t variant);  // ket points per lane; 0 if invalid
// Butterfly sweep (reps 1..3) over a tile list whose length a.tile_count
// holds in device memory: one persistent launch, no host read of the count.
hipError_t launch_sweep_butterfly_counted(const SweepArgs& a, int32_t reps, int32_t variant, hipStream_t stream);
// reps = 4..6: the environment split across 2, 8 or 32 lanes (sweep_split.hip).
hipError_t launch_sweep_split_args(const SweepArgs& a, int32_t reps, int32_t variant, hipStream_t stream);
int32_t split_blocks_per_tile(int32_t reps);  // blocks per 64 x 64 tile of the split sweep
// The fast (Section G) sweep for any supported reps.
inline hipError_t launch_sweep_fast(const SweepArgs& a, int32_t reps, int32_t variant, hipStream_t stream) {
  return reps <= 3 ? launch_sweep_butterfly_args(a, reps, variant, stream)
                   : launch_sweep_split_args(a, reps, variant, stream);
}
// Autotuned variant table (autotune.cpp).
// Tuned variant for (reps, n qubits, N points): N is the point count of a
// symmetric Gram, sqrt(2 Na Nb) for a rectangular one (the same pair count).
int32_t tuned_variant(int32_t reps, int32_t n, int64_t N);
void set_tuned_variant(int32_t reps, int32_t n, int64_t N, int32_t variant);
bool save_tuned_table();  // merge the table into the cache file; false on an I/O error
std::string tune_cache_path();  // the cache file in use ("" = none)
hipError_t autotune_run(int32_t reps, int32_t n, int64_t N, hipStream_t stream, int32_t* best, float* ms_out);
hipError_t launch_sweep_dense_args(const SweepArgs& a, int32_t reps, hipStream_t stream);
// State-vector engine (sv.hip).
constexpr int32_t kMaxSvQubits = 30;
constexpr int32_t kMaxSvReps = 16;
hipError_t launch_encode_sv(const double* X, int64_t N, int32_t n, int32_t reps, void* sv, hipStream_t stream);
hipError_t launch_sv_gram(const SweepArgs& a, const void* sv_a, const void* sv_b, int32_t n, hipStream_t stream);

}  // namespace qsvm
