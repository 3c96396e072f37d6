// Host side of the batched persistent sweep: validates the jobs, orders their
// work items longest-processing-time-first, uploads the job table, sizes the
// persistent grid from the kernel's occupancy, and optionally captures the
// launch (counter reset + persistent kernel) into a hipGraph for replay.

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/qsvm.h"
#include "batched.h"
#include "qsvm_internal.h"
#include "trace.h"
#include "refine.h"

struct qsvm_batch_plan {
  int device = -1;
  qsvm::BatchJob* d_jobs = nullptr;
  unsigned int* d_counter = nullptr;
  int32_t n_jobs = 0;
  int64_t total_items = 0;
  uint32_t grid = 0;
  qsvm::BatchShape shape;
  bool use_graph = false;
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t last_launch = nullptr;
  bool launched = false;
  // FP64 refinement after the persistent sweep, job by job
  std::vector<qsvm::BatchJob> host_jobs;
  double refine_above = 0.0;          // 0: automatic per job; negative: off
  uint32_t* d_refine = nullptr;       // [count, list of the largest job's tiles]
  int64_t refine_resident[4] = {0, 0, 0, 0};
};

namespace qsvm {

void destroy_plan(qsvm_batch_plan* p) {
  if (!p) return;
  if (p->launched && p->last_launch) (void)hipEventSynchronize(p->last_launch);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  if (p->last_launch) (void)hipEventDestroy(p->last_launch);
  if (p->d_jobs) (void)hipFree(p->d_jobs);
  if (p->d_counter) (void)hipFree(p->d_counter);
  if (p->d_refine) (void)hipFree(p->d_refine);
  delete p;
}

// The persistent sweep of every job, then each job's FP64 refinement of its
// tiles with an entry above the threshold (no allocation, no memset: the
// sequence can be captured in a graph).
hipError_t plan_enqueue(qsvm_batch_plan* p, hipStream_t s) {
  hipError_t e = launch_batch(p->shape, p->d_jobs, p->n_jobs, p->total_items, p->d_counter, p->grid, s);
  if (e != hipSuccess || p->refine_above < 0.0) return e;
  for (const BatchJob& j : p->host_jobs) {
    const double thresh = p->refine_above > 0.0 ? p->refine_above : auto_refine_threshold(j.args.n);
    if (thresh >= 1.0) continue;  // no entry of this job can need it
    e = launch_chunked(j.args, 1, [&](const SweepArgs& c) {
      return launch_refine(c, j.reps, thresh, p->d_refine + 1, p->d_refine, p->refine_resident[j.reps], s);
    });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Build the host job table; returns false with a message on invalid input.
bool build_jobs(const qsvm_job* jobs, int32_t n_jobs, int32_t renorm_every, int32_t diag_mode, const BatchShape& shape,
                std::vector<BatchJob>& out, int64_t& total, char* msg, size_t msg_len) {
  struct Entry {
    BatchJob job;
    double cost;
    int64_t items;
  };
  std::vector<Entry> es;
  es.reserve(size_t(n_jobs));
  for (int32_t q = 0; q < n_jobs; ++q) {
    const qsvm_job& J = jobs[q];
    if (!J.mps || !J.K) {
      snprintf(msg, msg_len, "job %d: mps or K is NULL", q);
      return false;
    }
    if (J.N < 1 || J.N > (int64_t(1) << 31) - 1 || J.n_qubits < 1 || J.n_qubits > 65535 || J.reps < 1 ||
        J.reps > 3 || J.ldk < J.N || (reinterpret_cast<uintptr_t>(J.mps) % 16) != 0) {
      snprintf(msg, msg_len, "job %d: invalid shape (N=%lld n=%d reps=%d ldk=%lld) or misaligned mps", q,
               (long long)J.N, J.n_qubits, J.reps, (long long)J.ldk);
      return false;
    }
    Entry e{};
    SweepArgs& a = e.job.args;
    a.gen_a = a.gen_b = static_cast<const float4*>(J.mps);  // butterfly sweep: no dense tensors
    a.K = J.K;
    a.log_k = J.log_k;
    a.Na = a.Nb = J.N;
    a.ldk = J.ldk;
    a.row_begin = 0;
    a.row_end = J.N;
    a.n = J.n_qubits;
    a.renorm_every = renorm_every;
    a.sym = 1;
    a.diag_mode = diag_mode;
    a.tile_row0 = 0;
    a.tiles_b = a.tile_rows = int32_t((J.N + kTile - 1) / kTile);
    a.blocks_per_tile = batch_blocks_per_tile(shape, J.reps);
    const int64_t T = a.tiles_b;
    e.items = (T * (T + 1) / 2) * a.blocks_per_tile;
    a.num_blocks = 0;  // unused by the persistent kernel
    e.job.reps = J.reps;
    e.cost = batch_item_cost(shape, J.reps, J.n_qubits);
    es.push_back(e);
  }
  // longest processing time first: most expensive items at the head of the queue
  std::stable_sort(es.begin(), es.end(), [](const Entry& x, const Entry& y) { return x.cost > y.cost; });
  total = 0;
  out.clear();
  for (Entry& e : es) {
    e.job.item_begin = total;
    total += e.items;
    out.push_back(e.job);
  }
  return true;
}

}  // namespace qsvm

extern "C" {

qsvm_status qsvm_batch_plan_create(const qsvm_job* jobs, int32_t n_jobs, const qsvm_batch_opts* opts,
                                   qsvm_batch_plan** plan_out);
qsvm_status qsvm_batch_plan_launch(qsvm_batch_plan* plan, void* stream);
qsvm_status qsvm_batch_plan_destroy(qsvm_batch_plan* plan);
qsvm_status qsvm_batch_plan_info(const qsvm_batch_plan* plan, int64_t* total_items, int32_t* grid_blocks,
                                 int32_t* uses_graph);
qsvm_status qsvm_batch_plan_shape(const qsvm_batch_plan* plan, int32_t* item_pi2, int32_t* item_pi3);

}  // extern "C"

namespace qsvm {
qsvm_status api_fail(qsvm_status s, const char* msg);
qsvm_status api_ok();
qsvm_status api_hip(hipError_t e, const char* what);
bool api_injected_failure();
}  // namespace qsvm

extern "C" qsvm_status qsvm_batch_plan_create(const qsvm_job* jobs, int32_t n_jobs, const qsvm_batch_opts* opts,
                                              qsvm_batch_plan** plan_out) {
  QSVM_TRACE_RANGE("qsvm_batch_plan_create");
  using namespace qsvm;
  char msg[256];
  if (!plan_out) return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_batch_plan_create: plan is NULL");
  *plan_out = nullptr;
  if (!jobs || n_jobs < 1) return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_batch_plan_create: no jobs");
  qsvm_batch_opts o{};
  if (opts) o = *opts;
  if (o.renorm_every < 0 || o.renorm_every > kMaxRenorm)
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_batch_plan_create: renorm_every outside [0, 16]");
  if (o.diag_mode != 0 && o.diag_mode != 1)
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_batch_plan_create: diag_mode must be 0 or 1");
  if (o.use_graph != 0 && o.use_graph != 1)
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_batch_plan_create: use_graph must be 0 or 1");
  if (o.grid_blocks < 0 || o.grid_blocks > (1 << 24) - 8)
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_batch_plan_create: grid_blocks outside [0, 2^24 - 8]");
  if (!(o.refine_above == o.refine_above))
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_batch_plan_create: refine_above is NaN");
  for (int32_t q = 0; q < n_jobs; ++q) {
    if (jobs[q].reps > 3) {
      snprintf(msg, sizeof msg,
               "qsvm_batch_plan_create: job %d: reps = %d > 3 is not supported in a batch plan", q, jobs[q].reps);
      return api_fail(QSVM_ERR_UNSUPPORTED, msg);
    }
  }
  // work-item shape: forced by opts, else the tuned single-Gram variant of the
  // costliest job of each reps (its ket points per lane)
  BatchShape shape;
  if (o.item_pi2 != 0 || o.item_pi3 != 0) {
    shape.pi2 = o.item_pi2 ? o.item_pi2 : shape.pi2;
    shape.pi3 = o.item_pi3 ? o.item_pi3 : shape.pi3;
    if (!batch_shape_supported(shape))
      return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_batch_plan_create: item_pi2 must be 0, 2 or 4 and item_pi3 0 or 1");
  } else {
    for (int r = 2; r <= 3; ++r) {
      double best = -1.0;
      int32_t n_best = 0;
      int64_t N_best = 0;
      for (int32_t q = 0; q < n_jobs; ++q) {
        if (jobs[q].reps != r || jobs[q].N < 1 || jobs[q].n_qubits < 1) continue;
        const double cost = double(jobs[q].N) * double(jobs[q].N) * double(jobs[q].n_qubits);
        if (cost > best) {
          best = cost;
          n_best = jobs[q].n_qubits;
          N_best = jobs[q].N;
        }
      }
      if (n_best == 0) continue;
      // a tuned shape the persistent kernel cannot hold (two reps = 3 points
      // per lane) keeps the default
      const int32_t pi = butterfly_variant_pi(r, tuned_variant(r, n_best, N_best));
      BatchShape t = shape;
      (r == 2 ? t.pi2 : t.pi3) = pi;
      if (batch_shape_supported(t)) shape = t;
    }
  }
  std::vector<BatchJob> table;
  int64_t total = 0;
  if (!build_jobs(jobs, n_jobs, o.renorm_every ? o.renorm_every : kDefaultRenorm, o.diag_mode, shape, table, total,
                  msg, sizeof msg))
    return api_fail(QSVM_ERR_INVALID_ARG, msg);
  if (api_injected_failure()) return api_fail(QSVM_ERR_HIP, "qsvm_batch_plan_create: injected launch failure (QSVM_FAULT_INJECT=launch)");

  qsvm_batch_plan* p = new (std::nothrow) qsvm_batch_plan();
  if (!p) return api_fail(QSVM_ERR_HIP, "qsvm_batch_plan_create: out of host memory");
  hipError_t e = hipGetDevice(&p->device);
  int cus = 0, per_cu = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e == hipSuccess) e = batch_kernel_occupancy(shape, &per_cu);
  if (e != hipSuccess) {
    destroy_plan(p);
    return api_hip(e, "qsvm_batch_plan_create");
  }
  p->grid = o.grid_blocks ? uint32_t(o.grid_blocks) : uint32_t(std::max(1, cus) * std::max(1, per_cu));
  if (total + int64_t(p->grid) >= (int64_t(1) << 31)) {
    destroy_plan(p);
    return api_fail(QSVM_ERR_UNSUPPORTED, "qsvm_batch_plan_create: more than 2^31 work items");
  }
  p->n_jobs = n_jobs;
  p->shape = shape;
  p->total_items = total;
  p->host_jobs = table;
  p->refine_above = o.refine_above;
  int64_t max_tiles = 1;
  for (const BatchJob& j : table) max_tiles = std::max(max_tiles, std::min(launch_tiles(j.args), kMaxGridBlocks));
  if (p->refine_above >= 0.0) {
    for (int r = 1; r <= 3 && e == hipSuccess; ++r) e = refine_resident_blocks(r, &p->refine_resident[r]);
    if (e == hipSuccess) e = hipMalloc(&p->d_refine, sizeof(uint32_t) * size_t(max_tiles + 1));
  }
  if (e == hipSuccess) e = hipMalloc(&p->d_jobs, sizeof(BatchJob) * table.size());
  if (e == hipSuccess) e = hipMalloc(&p->d_counter, sizeof(unsigned int));
  if (e == hipSuccess) e = hipMemcpy(p->d_jobs, table.data(), sizeof(BatchJob) * table.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->last_launch, hipEventDisableTiming);
  if (e == hipSuccess && o.use_graph) {
    p->use_graph = true;
    e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t le = plan_enqueue(p, p->capture_stream);
      e = hipStreamEndCapture(p->capture_stream, &p->graph);
      if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  }
  if (e != hipSuccess) {
    destroy_plan(p);
    return api_hip(e, "qsvm_batch_plan_create");
  }
  *plan_out = p;
  return api_ok();
}

extern "C" qsvm_status qsvm_batch_plan_launch(qsvm_batch_plan* p, void* stream) {
  QSVM_TRACE_RANGE("qsvm_batch_plan_launch");
  using namespace qsvm;
  if (!p) return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_batch_plan_launch: plan is NULL");
  if (api_injected_failure()) return api_fail(QSVM_ERR_HIP, "qsvm_batch_plan_launch: injected launch failure (QSVM_FAULT_INJECT=launch)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = p->use_graph ? hipGraphLaunch(p->exec, s) : plan_enqueue(p, s);
  if (e == hipSuccess) e = hipEventRecord(p->last_launch, s);
  if (e == hipSuccess) p->launched = true;
  return api_hip(e, "qsvm_batch_plan_launch");
}

extern "C" qsvm_status qsvm_batch_plan_destroy(qsvm_batch_plan* p) {
  qsvm::destroy_plan(p);
  return qsvm::api_ok();
}

extern "C" qsvm_status qsvm_batch_plan_shape(const qsvm_batch_plan* p, int32_t* item_pi2, int32_t* item_pi3) {
  using namespace qsvm;
  if (!p) return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_batch_plan_shape: plan is NULL");
  if (item_pi2) *item_pi2 = p->shape.pi2;
  if (item_pi3) *item_pi3 = p->shape.pi3;
  return api_ok();
}

extern "C" qsvm_status qsvm_batch_plan_info(const qsvm_batch_plan* p, int64_t* total_items, int32_t* grid_blocks,
                                            int32_t* uses_graph) {
  using namespace qsvm;
  if (!p) return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_batch_plan_info: plan is NULL");
  if (total_items) *total_items = p->total_items;
  if (grid_blocks) *grid_blocks = int32_t(p->grid);
  if (uses_graph) *uses_graph = p->use_graph ? 1 : 0;
  return api_ok();
}
