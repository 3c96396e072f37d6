// Device job table and launch helpers of the batched persistent sweep.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sweep_common.h"

namespace qsvm {

// One symmetric Gram job as the persistent kernel reads it.
struct BatchJob {
  SweepArgs args;      // the job's sweep arguments (sym = 1, blocks_per_tile set)
  int32_t reps;
  int32_t pad;
  int64_t item_begin;  // first queue item of this job (jobs sorted by it)
};

// Work-item shape of a plan: ket points per lane of the reps = 2 and reps = 3
// items (reps = 1 items use 4).  Supported: pi2 in {2, 4}, pi3 = 1.
struct BatchShape {
  int32_t pi2 = 2;
  int32_t pi3 = 1;
};

bool batch_shape_supported(const BatchShape& s);
int batch_pi(const BatchShape& s, int reps);
int batch_blocks_per_tile(const BatchShape& s, int reps);
double batch_item_cost(const BatchShape& s, int reps, int32_t n);
hipError_t batch_kernel_occupancy(const BatchShape& s, int* blocks_per_cu);
hipError_t launch_batch(const BatchShape& s, const BatchJob* d_jobs, int32_t n_jobs, int64_t total_items,
                        unsigned int* d_counter, uint32_t grid, hipStream_t stream);

}  // namespace qsvm
