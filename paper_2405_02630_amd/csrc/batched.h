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

int batch_blocks_per_tile(int reps);
double batch_item_cost(int reps, int32_t n);
hipError_t batch_kernel_occupancy(int* blocks_per_cu);
hipError_t launch_batch(const BatchJob* d_jobs, int32_t n_jobs, int64_t total_items,
                        unsigned int* d_counter, uint32_t grid, hipStream_t stream);

}  // namespace qsvm
