// Batched Gram jobs in one persistent launch.
//
// The paper keeps contractions flowing without host round trips by reusing
// one contraction path and running contractions concurrently while tensors
// stay on the device (§4.1).  Here many independent symmetric Gram jobs of
// different sizes (n, N) and depths (reps) are drained by one persistent
// kernel: every job is cut into the same work items the single-Gram sweep
// uses (one block = 4 waves = 4 groups of PI ket points x 64 bra points of
// one tile; PI per reps chosen by the plan from the tuned variants), the
// items of all jobs form one queue ordered by decreasing cost
// per item (longest-processing-time-first), and each resident block pops the
// next item with an atomic counter until the queue is empty.  A job's reps
// selects the code path per item (wave-uniform).  The counter is cleared by a
// one-thread kernel launched just before (no memset node, so the pair can be
// captured in a hipGraph and replayed).

#include "../../include/qsvm.h"
#include "batched.h"
#include "sweep_butterfly_item.h"

namespace qsvm {
namespace {

constexpr int kBatchWaves = 4;  // target waves per SIMD of the persistent kernel

__global__ void reset_counter(unsigned int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

// PI2, PI3: ket points per lane of the reps = 2 and reps = 3 items (reps = 1
// items use 4); the plan picks them from the tuned single-Gram variants.
template <int PI2, int PI3>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kBatchWaves, 8)))
batched_kernel(const BatchJob* __restrict__ jobs, int32_t n_jobs, int64_t total_items,
               unsigned int* __restrict__ counter) {
  // total_items + gridDim.x < 2^31 (checked on the host), so the counter and
  // item indices fit in 32 bits
  __shared__ unsigned int item_s;
  for (;;) {
    if (threadIdx.x == 0) item_s = atomicAdd(counter, 1u);
    __syncthreads();
    const int64_t u = int64_t(uint32_t(__builtin_amdgcn_readfirstlane(int(item_s))));
    __syncthreads();  // every wave has read item_s before thread 0 overwrites it
    if (u >= total_items) return;
    // job of item u: last job with item_begin <= u (jobs sorted by item_begin)
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (jobs[mid].item_begin <= u) lo = mid; else hi = mid - 1;
    }
    const SweepArgs a = jobs[lo].args;
    const int reps = jobs[lo].reps;
    const int64_t local = u - jobs[lo].item_begin;
    const uint32_t bpt = uint32_t(a.blocks_per_tile);
    const uint32_t tile = uint32_t(local / bpt);
    const uint32_t sub = uint32_t(local % bpt);
    int32_t ti, tj;
    decode_tile(a, tile, ti, tj);  // the job table holds no tile lists
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t j0 = int64_t(tj) * kTile;
    if (reps == 2) {
      butterfly_item<2, PI2>(a, int64_t(ti) * kTile + (int64_t(sub) * 4 + wave) * PI2, j0);
    } else if (reps == 3) {
      butterfly_item<3, PI3>(a, int64_t(ti) * kTile + (int64_t(sub) * 4 + wave) * PI3, j0);
    } else {
      butterfly_item<1, 4>(a, int64_t(ti) * kTile + (int64_t(sub) * 4 + wave) * 4, j0);
    }
  }
}

// Kernel instance for a choice of ket points per lane: PI2 in {2, 4}; PI3 = 1
// only (at the kernel's 4 waves per SIMD, 128 VGPRs, two reps = 3
// environments per lane spill ~860 VGPRs).
template <class F>
hipError_t with_kernel(const BatchShape& s, F f) {
  if (s.pi2 == 2 && s.pi3 == 1) return f(batched_kernel<2, 1>);
  if (s.pi2 == 4 && s.pi3 == 1) return f(batched_kernel<4, 1>);
  return hipErrorInvalidValue;
}

}  // namespace

int batch_pi(const BatchShape& s, int reps) { return reps == 1 ? 4 : (reps == 2 ? s.pi2 : s.pi3); }

int batch_blocks_per_tile(const BatchShape& s, int reps) { return kTile / (4 * batch_pi(s, reps)); }

// Host-side cost model of one item: pairs x sites x operations per site.
double batch_item_cost(const BatchShape& s, int reps, int32_t n) {
  const double per_site = double(2 * reps - 1) * double(1 << (2 * reps - 2)) * 16.0 + 12.0;
  return double(4 * batch_pi(s, reps) * kTile) * double(n) * per_site;
}

bool batch_shape_supported(const BatchShape& s) { return (s.pi2 == 2 || s.pi2 == 4) && s.pi3 == 1; }

hipError_t batch_kernel_occupancy(const BatchShape& s, int* blocks_per_cu) {
  return with_kernel(s, [&](auto k) { return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, 256, 0); });
}

hipError_t launch_batch(const BatchShape& s, const BatchJob* d_jobs, int32_t n_jobs, int64_t total_items,
                        unsigned int* d_counter, uint32_t grid, hipStream_t stream) {
  hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, stream, d_counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return with_kernel(s, [&](auto k) {
    hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, stream, d_jobs, n_jobs, total_items, d_counter);
    return hipGetLastError();
  });
}

}  // namespace qsvm
