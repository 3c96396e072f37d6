// C-ABI layer of libqsvm.so: argument validation, defaults and dispatch to the
// HIP kernels.  Every check runs on the host before any HIP call, so a
// rejected call enqueues nothing and touches no device state.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <string>

#include "../../include/qsvm.h"
#include "qsvm_internal.h"
#include "trace.h"
#include "refine.h"
#include "sweep_common.h"

namespace {

thread_local std::string g_last_error;

constexpr int64_t kMaxN = (int64_t(1) << 31) - 1;
constexpr int32_t kMaxQubits = 65535;

qsvm_status fail(qsvm_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

qsvm_status fail(qsvm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

qsvm_status ok() {
  g_last_error.clear();
  return QSVM_OK;
}

qsvm_status check_shape(int64_t N, int32_t n, int32_t reps, const char* what) {
  if (N < 1 || N > kMaxN) return fail(QSVM_ERR_INVALID_ARG, "%s: N = %lld outside [1, 2^31-1]", what, (long long)N);
  if (n < 1 || n > kMaxQubits) return fail(QSVM_ERR_INVALID_ARG, "%s: n_qubits = %d outside [1, 65535]", what, n);
  if (reps < 1) return fail(QSVM_ERR_INVALID_ARG, "%s: reps = %d must be >= 1", what, reps);
  if (reps > qsvm::kMaxReps)
    return fail(QSVM_ERR_UNSUPPORTED, "%s: reps = %d > 6 (bond dimension above 64) is not supported", what, reps);
  return QSVM_OK;
}

// Host-forced failure for tests of the error path: QSVM_FAULT_INJECT=launch
// makes every call that passed validation return QSVM_ERR_HIP instead of
// launching.
bool injected_launch_failure() {
  const char* v = getenv("QSVM_FAULT_INJECT");
  return v && strcmp(v, "launch") == 0;
}

qsvm_status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return ok();
  return fail(QSVM_ERR_HIP, "%s: HIP error %d (%s)", what, int(e), hipGetErrorString(e));
}

struct Opts {
  int32_t renorm_every = qsvm::kDefaultRenorm;
  int32_t sweep = QSVM_SWEEP_BUTTERFLY;
  int32_t diag_mode = 0;
  int32_t variant = 0;
  int64_t row_begin = 0, row_end = 0;
  double* log_k = nullptr;
  double refine_above = 0.0;  // 0: automatic (qsvm::auto_refine_threshold); negative: no refinement
  const void* dense_a = nullptr;  // dense tensors of the sets (dense sweep only)
  const void* dense_b = nullptr;
};

qsvm_status read_opts(const qsvm_gram_opts* o, int64_t rows, Opts& out, const char* what) {
  out = Opts{};
  out.row_end = rows;
  if (!o) return QSVM_OK;
  if (o->renorm_every < 0 || o->renorm_every > qsvm::kMaxRenorm)
    return fail(QSVM_ERR_INVALID_ARG, "%s: renorm_every = %d outside [0, %d]", what, o->renorm_every, qsvm::kMaxRenorm);
  if (o->renorm_every) out.renorm_every = o->renorm_every;
  if (o->sweep < QSVM_SWEEP_AUTO || o->sweep > QSVM_SWEEP_DENSE)
    return fail(QSVM_ERR_INVALID_ARG, "%s: unknown sweep kind %d", what, o->sweep);
  out.sweep = (o->sweep == QSVM_SWEEP_DENSE) ? QSVM_SWEEP_DENSE : QSVM_SWEEP_BUTTERFLY;
  if (o->diag_mode != 0 && o->diag_mode != 1)
    return fail(QSVM_ERR_INVALID_ARG, "%s: diag_mode = %d must be 0 or 1", what, o->diag_mode);
  out.diag_mode = o->diag_mode;
  if (o->variant < 0 || o->variant > qsvm::kButterflyVariants)
    return fail(QSVM_ERR_INVALID_ARG, "%s: variant = %d outside [0, %d]", what, o->variant, qsvm::kButterflyVariants);
  out.variant = o->variant;
  if (o->row_begin != 0 || o->row_end != 0) {
    if (o->row_begin < 0 || o->row_end < o->row_begin || o->row_end > rows)
      return fail(QSVM_ERR_INVALID_ARG, "%s: row range [%lld, %lld) outside [0, %lld]", what,
                  (long long)o->row_begin, (long long)o->row_end, (long long)rows);
    out.row_begin = o->row_begin;
    out.row_end = o->row_end;
  }
  out.log_k = o->log_k;
  if (!(o->refine_above == o->refine_above))  // NaN
    return fail(QSVM_ERR_INVALID_ARG, "%s: refine_above is NaN", what);
  if (o->refine_above != 0.0) out.refine_above = o->refine_above;
  out.dense_a = o->dense_a;
  out.dense_b = o->dense_b ? o->dense_b : o->dense_a;
  if (out.sweep == QSVM_SWEEP_DENSE) {
    if (!out.dense_a)
      return fail(QSVM_ERR_INVALID_ARG, "%s: the dense sweep needs opts.dense_a (tensors from qsvm_encode_dense)", what);
    if ((reinterpret_cast<uintptr_t>(out.dense_a) | reinterpret_cast<uintptr_t>(out.dense_b)) % 16 != 0)
      return fail(QSVM_ERR_INVALID_ARG, "%s: dense tensors are not 16-byte aligned", what);
  }
  return QSVM_OK;
}

// Blocks of the refinement kernel resident on the current device, cached per
// device and reps.
hipError_t resident_refine_blocks(int32_t reps, int64_t* out) {
  static std::atomic<int64_t> cache[64][qsvm::kMaxReps + 1];  // zero-initialised (static storage)
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const bool cacheable = dev >= 0 && dev < 64 && reps >= 1 && reps <= qsvm::kMaxReps;
  if (cacheable) {
    const int64_t c = cache[dev][reps].load(std::memory_order_relaxed);
    if (c > 0) {
      *out = c;
      return hipSuccess;
    }
  }
  e = qsvm::refine_resident_blocks(reps, out);
  if (e == hipSuccess && cacheable) cache[dev][reps].store(*out, std::memory_order_relaxed);
  return e;
}

// The refinement threshold a call uses: the automatic one for 0.  The
// refinement runs only for thresholds in (0, 1) (negative: off; >= 1: no entry
// can need it).
double effective_refine_threshold(double refine_above, int32_t n) {
  return refine_above == 0.0 ? qsvm::auto_refine_threshold(n) : refine_above;
}
bool refine_runs(double thresh) { return thresh > 0.0 && thresh < 1.0; }

// uint32 entries of the refinement's workspace ([count, tile list...]) for the
// tiles of `a`: launch_chunked issues at most kMaxGridBlocks tiles per chunk
// and the chunks reuse the workspace in stream order.
int64_t refine_workspace_entries(const qsvm::SweepArgs& a) {
  const int64_t tiles = qsvm::launch_tiles(a);
  if (tiles <= 0) return 0;
  return (tiles < qsvm::kMaxGridBlocks ? tiles : qsvm::kMaxGridBlocks) + 1;
}

// Where the refinement's workspace comes from: a stream-ordered temporary
// (get == nullptr) or memory the caller obtains without allocating.
struct WorkspaceSource {
  hipError_t (*get)(uint32_t** ptr) = nullptr;
  int64_t entries = 0;  // capacity of what `get` returns
};

// FP64 refinement of the tiles of `a` (the tiles one Gram call swept) whose
// largest entry exceeds the threshold, chunk by chunk like the sweeps.
hipError_t refine_tiles(const qsvm::SweepArgs& a, int32_t reps, double refine_above, hipStream_t stream,
                        const WorkspaceSource& src) {
  const double thresh = effective_refine_threshold(refine_above, a.n);
  if (!refine_runs(thresh)) return hipSuccess;
  const int64_t need = refine_workspace_entries(a);
  if (need <= 0) return hipSuccess;
  int64_t resident = 0;
  hipError_t e = resident_refine_blocks(reps, &resident);
  if (e != hipSuccess) return e;
  uint32_t* ws = nullptr;  // [count, list...]
  if (src.get) {
    if (need > src.entries) return hipErrorInvalidValue;  // callers validate this first
    e = src.get(&ws);
  } else {
    e = hipMallocAsync(reinterpret_cast<void**>(&ws), size_t(need) * sizeof(uint32_t), stream);
  }
  if (e != hipSuccess) return e;
  e = qsvm::launch_chunked(a, 1, [&](const qsvm::SweepArgs& c) {
    return qsvm::launch_refine(c, reps, thresh, ws + 1, ws, resident, stream);
  });
  const hipError_t f = src.get ? hipSuccess : hipFreeAsync(ws, stream);
  return e != hipSuccess ? e : f;
}

// Variant for a launch: forced by opts, else the tuned table (default 0) at
// the symmetric point count with the launch's pair count.
int32_t pick_variant(const Opts& o, int32_t reps, int32_t n, double pairs) {
  if (o.variant > 0) return o.variant - 1;
  return qsvm::tuned_variant(reps, n, int64_t(sqrt(2.0 * (pairs > 1.0 ? pairs : 1.0)) + 0.5));
}

qsvm_status run_gram(const void* mps_a, int64_t Na, const void* mps_b, int64_t Nb, int32_t n,
                     int32_t reps, double* K, int64_t ldk, const Opts& o, bool sym, void* stream,
                     const char* what, const WorkspaceSource& src = WorkspaceSource{}) {
  using qsvm::kTile;
  if (o.sweep == QSVM_SWEEP_DENSE && reps > 3)
    return fail(QSVM_ERR_UNSUPPORTED, "%s: the dense sweep supports reps <= 3", what);
  // the sweeps launch whole rows of tiles (at most 16 blocks per tile, 32,
  // 128 and 512 in the split sweep of reps 4, 5 and 6), so one row must fit
  // one launch
  const int64_t tiles_b = (Nb + kTile - 1) / kTile;
  if (tiles_b * (reps >= 4 ? qsvm::split_blocks_per_tile(reps) : 16) > qsvm::kMaxGridBlocks)
    return fail(QSVM_ERR_UNSUPPORTED, "%s: Nb = %lld: one row of %lld tiles exceeds one launch", what, (long long)Nb,
                (long long)tiles_b);
  if (o.row_end <= o.row_begin) return ok();  // empty row range: nothing to do
  qsvm::SweepArgs a{};
  a.gen_a = static_cast<const float4*>(mps_a);
  a.gen_b = static_cast<const float4*>(mps_b);
  a.dense_a = static_cast<const float2*>(o.dense_a);
  a.dense_b = static_cast<const float2*>(o.dense_b);
  a.K = K;
  a.log_k = o.log_k;
  a.Na = Na;
  a.Nb = Nb;
  a.ldk = ldk;
  a.row_begin = o.row_begin;
  a.row_end = o.row_end;
  a.n = n;
  a.renorm_every = o.renorm_every;
  a.sym = sym ? 1 : 0;
  a.diag_mode = o.diag_mode;
  a.tile_row0 = int32_t(o.row_begin / kTile);
  a.tile_rows = int32_t((o.row_end - 1) / kTile) - a.tile_row0 + 1;
  a.tiles_b = int32_t(tiles_b);
  if (src.get && refine_runs(effective_refine_threshold(o.refine_above, n)) &&
      refine_workspace_entries(a) > src.entries)
    return fail(QSVM_ERR_SIZE, "%s: the refinement needs a %lld-entry tile list, the static workspace holds %lld",
                what, (long long)refine_workspace_entries(a), (long long)src.entries);
  if (injected_launch_failure()) return fail(QSVM_ERR_HIP, "%s: injected launch failure (QSVM_FAULT_INJECT=launch)", what);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = (o.sweep == QSVM_SWEEP_DENSE) ? qsvm::launch_sweep_dense_args(a, reps, s)
                                                : qsvm::launch_sweep_fast(
                                                      a, reps, pick_variant(o, reps, n, sym ? 0.5 * double(Na) * double(Na)
                                                                                            : double(Na) * double(Nb)),
                                                      s);
  if (e == hipSuccess) e = refine_tiles(a, reps, o.refine_above, s, src);
  return hip_status(e, what);
}

// Symmetric Gram over a list of (ti, tj) tiles: n_tiles entries, or, with
// tile_count, at most n_tiles entries, the count read on the device.
qsvm_status gram_tile_list(const void* mps, int64_t N, int32_t n_qubits, int32_t reps, const int32_t* tiles,
                           const int32_t* tile_count, int64_t n_tiles, double* K, int64_t ldk,
                           const qsvm_gram_opts* opts, void* stream, const char* what) {
  qsvm_status s = check_shape(N, n_qubits, reps, what);
  if (s != QSVM_OK) return s;
  if (!mps || !K || !tiles) return fail(QSVM_ERR_INVALID_ARG, "%s: mps, tiles or K is NULL", what);
  if (ldk < N) return fail(QSVM_ERR_INVALID_ARG, "%s: ldk = %lld < N = %lld", what, (long long)ldk, (long long)N);
  if (reinterpret_cast<uintptr_t>(mps) % 16 != 0) return fail(QSVM_ERR_INVALID_ARG, "%s: mps is not 16-byte aligned", what);
  const int64_t T = (N + qsvm::kTile - 1) / qsvm::kTile;
  if (n_tiles < 0 || n_tiles > T * (T + 1) / 2)
    return fail(QSVM_ERR_INVALID_ARG, "%s: n_tiles = %lld outside [0, %lld]", what, (long long)n_tiles, (long long)(T * (T + 1) / 2));
  if (n_tiles > INT32_MAX)
    return fail(QSVM_ERR_UNSUPPORTED, "%s: n_tiles = %lld above 2^31-1", what, (long long)n_tiles);
  Opts o;
  s = read_opts(opts, N, o, what);
  if (s != QSVM_OK) return s;
  if (o.row_begin != 0 || o.row_end != N) return fail(QSVM_ERR_INVALID_ARG, "%s: row ranges do not apply to tile lists", what);
  if (o.sweep == QSVM_SWEEP_DENSE && reps > 3)
    return fail(QSVM_ERR_UNSUPPORTED, "%s: the dense sweep supports reps <= 3", what);
  if (tile_count) {
    if (o.sweep == QSVM_SWEEP_DENSE || reps > 3)
      return fail(QSVM_ERR_UNSUPPORTED, "%s: a device-resident tile count needs the butterfly sweep (reps <= 3)", what);
    if (n_tiles > qsvm::kMaxGridBlocks)
      return fail(QSVM_ERR_UNSUPPORTED, "%s: max_tiles = %lld above %lld", what, (long long)n_tiles,
                  (long long)qsvm::kMaxGridBlocks);
  }
  if (n_tiles == 0) return ok();
  if (injected_launch_failure()) return fail(QSVM_ERR_HIP, "%s: injected launch failure (QSVM_FAULT_INJECT=launch)", what);
  qsvm::SweepArgs a{};
  a.gen_a = a.gen_b = static_cast<const float4*>(mps);
  a.dense_a = static_cast<const float2*>(o.dense_a);
  a.dense_b = static_cast<const float2*>(o.dense_a);  // one set
  a.K = K;
  a.log_k = o.log_k;
  a.Na = a.Nb = N;
  a.ldk = ldk;
  a.row_begin = 0;
  a.row_end = N;
  a.n = n_qubits;
  a.renorm_every = o.renorm_every;
  a.sym = 1;
  a.diag_mode = o.diag_mode;
  a.tile_row0 = 0;
  a.tile_rows = int32_t(n_tiles);  // list length (capacity when the count is on the device)
  a.tiles_b = int32_t(T);
  a.tile_list = tiles;
  a.tile_count = tile_count;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int32_t variant = pick_variant(o, reps, n_qubits, double(n_tiles) * qsvm::kTile * qsvm::kTile);
  hipError_t e = tile_count                      ? qsvm::launch_sweep_butterfly_counted(a, reps, variant, st)
                 : (o.sweep == QSVM_SWEEP_DENSE) ? qsvm::launch_sweep_dense_args(a, reps, st)
                                                 : qsvm::launch_sweep_fast(a, reps, variant, st);
  if (e == hipSuccess) e = refine_tiles(a, reps, o.refine_above, st, WorkspaceSource{});
  return hip_status(e, what);
}

qsvm_status gram_sym(const void* mps, int64_t N, int32_t n_qubits, int32_t reps, double* K, int64_t ldk,
                     const qsvm_gram_opts* opts, void* stream, const char* what, const WorkspaceSource& src) {
  if (!mps) return fail(QSVM_ERR_INVALID_ARG, "%s: mps is NULL", what);
  if (!K) return fail(QSVM_ERR_INVALID_ARG, "%s: K is NULL", what);
  qsvm_status s = check_shape(N, n_qubits, reps, what);
  if (s != QSVM_OK) return s;
  if (ldk < N) return fail(QSVM_ERR_INVALID_ARG, "%s: ldk = %lld < N = %lld", what, (long long)ldk, (long long)N);
  if (reinterpret_cast<uintptr_t>(mps) % 16 != 0) return fail(QSVM_ERR_INVALID_ARG, "%s: mps is not 16-byte aligned", what);
  Opts o;
  s = read_opts(opts, N, o, what);
  if (s != QSVM_OK) return s;
  o.dense_b = o.dense_a;  // one set
  return run_gram(mps, N, mps, N, n_qubits, reps, K, ldk, o, true, stream, what, src);
}

}  // namespace

namespace qsvm {
// Status helpers shared with the batch-plan translation unit.
qsvm_status api_fail(qsvm_status s, const char* msg) { return fail(s, "%s", msg); }
qsvm_status api_ok() { return ok(); }
qsvm_status api_hip(hipError_t e, const char* what) { return hip_status(e, what); }
bool api_injected_failure() { return injected_launch_failure(); }

// qsvm_gram_sym with the refinement's tile list taken from `get_ws` (at most
// ws_entries uint32 entries) instead of a stream-ordered temporary; sizes that
// need more are rejected with QSVM_ERR_SIZE before anything is enqueued, and
// `get_ws` is called only when the refinement runs.
qsvm_status gram_sym_static_workspace(const void* mps, int64_t N, int32_t n_qubits, int32_t reps, double* K,
                                      int64_t ldk, const qsvm_gram_opts* opts, void* stream,
                                      hipError_t (*get_ws)(uint32_t**), int64_t ws_entries, const char* what) {
  WorkspaceSource src;
  src.get = get_ws;
  src.entries = ws_entries;
  return gram_sym(mps, N, n_qubits, reps, K, ldk, opts, stream, what, src);
}
}  // namespace qsvm

extern "C" {

size_t qsvm_mps_bytes(int64_t N, int32_t n_qubits, int32_t reps) {
  if (N < 1 || N > kMaxN || n_qubits < 1 || n_qubits > kMaxQubits || reps < 1 || reps > qsvm::kMaxReps) return 0;
  return size_t(qsvm::mps_total_bytes(N, n_qubits, reps));
}

qsvm_status qsvm_encode_mps(const double* X, int64_t N, int32_t n_qubits, int32_t reps, void* mps,
                            size_t mps_bytes, void* stream) {
  QSVM_TRACE_RANGE("qsvm_encode_mps");
  const char* what = "qsvm_encode_mps";
  qsvm_status s = check_shape(N, n_qubits, reps, what);
  if (s != QSVM_OK) return s;
  if (!X) return fail(QSVM_ERR_INVALID_ARG, "%s: X is NULL", what);
  if (!mps) return fail(QSVM_ERR_INVALID_ARG, "%s: mps is NULL", what);
  if (reinterpret_cast<uintptr_t>(mps) % 16 != 0) return fail(QSVM_ERR_INVALID_ARG, "%s: mps is not 16-byte aligned", what);
  if (reinterpret_cast<uintptr_t>(X) % 8 != 0) return fail(QSVM_ERR_INVALID_ARG, "%s: X is not 8-byte aligned", what);
  const size_t need = qsvm_mps_bytes(N, n_qubits, reps);
  if (mps_bytes < need)
    return fail(QSVM_ERR_SIZE, "%s: mps_bytes = %zu < %zu needed", what, mps_bytes, need);
  if (injected_launch_failure()) return fail(QSVM_ERR_HIP, "%s: injected launch failure (QSVM_FAULT_INJECT=launch)", what);
  return hip_status(qsvm::launch_encode(X, N, n_qubits, reps, mps, static_cast<hipStream_t>(stream)), what);
}

size_t qsvm_dense_bytes(int64_t N, int32_t n_qubits, int32_t reps) {
  if (N < 1 || N > kMaxN || n_qubits < 1 || n_qubits > kMaxQubits || reps < 1 || reps > qsvm::kMaxDenseReps) return 0;
  return size_t(qsvm::dense_bytes(N, n_qubits, reps));
}

qsvm_status qsvm_encode_dense(const double* X, int64_t N, int32_t n_qubits, int32_t reps, void* dense,
                              size_t dense_bytes, void* stream) {
  QSVM_TRACE_RANGE("qsvm_encode_dense");
  const char* what = "qsvm_encode_dense";
  qsvm_status s = check_shape(N, n_qubits, reps, what);
  if (s != QSVM_OK) return s;
  if (reps > qsvm::kMaxDenseReps)
    return fail(QSVM_ERR_UNSUPPORTED, "%s: dense tensors are written for reps <= %d", what, qsvm::kMaxDenseReps);
  if (!X) return fail(QSVM_ERR_INVALID_ARG, "%s: X is NULL", what);
  if (!dense) return fail(QSVM_ERR_INVALID_ARG, "%s: dense is NULL", what);
  if (reinterpret_cast<uintptr_t>(dense) % 16 != 0) return fail(QSVM_ERR_INVALID_ARG, "%s: dense is not 16-byte aligned", what);
  if (reinterpret_cast<uintptr_t>(X) % 8 != 0) return fail(QSVM_ERR_INVALID_ARG, "%s: X is not 8-byte aligned", what);
  const size_t need = qsvm_dense_bytes(N, n_qubits, reps);
  if (dense_bytes < need) return fail(QSVM_ERR_SIZE, "%s: dense_bytes = %zu < %zu needed", what, dense_bytes, need);
  if (injected_launch_failure()) return fail(QSVM_ERR_HIP, "%s: injected launch failure (QSVM_FAULT_INJECT=launch)", what);
  return hip_status(qsvm::launch_encode_dense(X, N, n_qubits, reps, dense, static_cast<hipStream_t>(stream)), what);
}

double qsvm_auto_refine_threshold(int32_t n_qubits) {
  return n_qubits < 1 ? 0.0 : qsvm::auto_refine_threshold(n_qubits);
}

qsvm_status qsvm_gram(const void* mps_a, int64_t Na, const void* mps_b, int64_t Nb, int32_t n_qubits,
                      int32_t reps, double* K, int64_t ldk, const qsvm_gram_opts* opts, void* stream) {
  QSVM_TRACE_RANGE("qsvm_gram");
  const char* what = "qsvm_gram";
  if (!mps_a || !mps_b) return fail(QSVM_ERR_INVALID_ARG, "%s: MPS buffer is NULL", what);
  if (!K) return fail(QSVM_ERR_INVALID_ARG, "%s: K is NULL", what);
  qsvm_status s = check_shape(Na, n_qubits, reps, what);
  if (s != QSVM_OK) return s;
  s = check_shape(Nb, n_qubits, reps, what);
  if (s != QSVM_OK) return s;
  if (ldk < Nb) return fail(QSVM_ERR_INVALID_ARG, "%s: ldk = %lld < Nb = %lld", what, (long long)ldk, (long long)Nb);
  if ((reinterpret_cast<uintptr_t>(mps_a) | reinterpret_cast<uintptr_t>(mps_b)) % 16 != 0)
    return fail(QSVM_ERR_INVALID_ARG, "%s: MPS buffer is not 16-byte aligned", what);
  Opts o;
  s = read_opts(opts, Na, o, what);
  if (s != QSVM_OK) return s;
  o.diag_mode = 0;
  return run_gram(mps_a, Na, mps_b, Nb, n_qubits, reps, K, ldk, o, false, stream, what);
}

qsvm_status qsvm_gram_sym(const void* mps, int64_t N, int32_t n_qubits, int32_t reps, double* K,
                          int64_t ldk, const qsvm_gram_opts* opts, void* stream) {
  QSVM_TRACE_RANGE("qsvm_gram_sym");
  return gram_sym(mps, N, n_qubits, reps, K, ldk, opts, stream, "qsvm_gram_sym", WorkspaceSource{});
}

qsvm_status qsvm_gram_sym_tiles(const void* mps, int64_t N, int32_t n_qubits, int32_t reps, const int32_t* tiles,
                                int64_t n_tiles, double* K, int64_t ldk, const qsvm_gram_opts* opts, void* stream) {
  QSVM_TRACE_RANGE("qsvm_gram_sym_tiles");
  return gram_tile_list(mps, N, n_qubits, reps, tiles, nullptr, n_tiles, K, ldk, opts, stream, "qsvm_gram_sym_tiles");
}

qsvm_status qsvm_gram_sym_tiles_dev(const void* mps, int64_t N, int32_t n_qubits, int32_t reps, const int32_t* tiles,
                                    const int32_t* tile_count, int64_t max_tiles, double* K, int64_t ldk,
                                    const qsvm_gram_opts* opts, void* stream) {
  QSVM_TRACE_RANGE("qsvm_gram_sym_tiles_dev");
  const char* what = "qsvm_gram_sym_tiles_dev";
  if (!tile_count) return fail(QSVM_ERR_INVALID_ARG, "%s: tile_count is NULL", what);
  return gram_tile_list(mps, N, n_qubits, reps, tiles, tile_count, max_tiles, K, ldk, opts, stream, what);
}

qsvm_status qsvm_gram_sym_pairs_dev(const void* mps, int64_t N, int32_t n_qubits, int32_t reps, const int32_t* pairs,
                                    const int32_t* pair_count, int64_t max_pairs, double* K, int64_t ldk,
                                    const qsvm_gram_opts* opts, void* stream) {
  QSVM_TRACE_RANGE("qsvm_gram_sym_pairs_dev");
  const char* what = "qsvm_gram_sym_pairs_dev";
  qsvm_status s = check_shape(N, n_qubits, reps, what);
  if (s != QSVM_OK) return s;
  if (!mps || !K || !pairs || !pair_count)
    return fail(QSVM_ERR_INVALID_ARG, "%s: mps, pairs, pair_count or K is NULL", what);
  if (ldk < N) return fail(QSVM_ERR_INVALID_ARG, "%s: ldk = %lld < N = %lld", what, (long long)ldk, (long long)N);
  if (reinterpret_cast<uintptr_t>(mps) % 16 != 0) return fail(QSVM_ERR_INVALID_ARG, "%s: mps is not 16-byte aligned", what);
  if (max_pairs < 0 || max_pairs > (int64_t(1) << 40))
    return fail(QSVM_ERR_INVALID_ARG, "%s: max_pairs = %lld outside [0, 2^40]", what, (long long)max_pairs);
  Opts o;
  s = read_opts(opts, N, o, what);
  if (s != QSVM_OK) return s;
  if (o.row_begin != 0 || o.row_end != N) return fail(QSVM_ERR_INVALID_ARG, "%s: row ranges do not apply to pair lists", what);
  if (max_pairs == 0) return ok();
  if (injected_launch_failure()) return fail(QSVM_ERR_HIP, "%s: injected launch failure (QSVM_FAULT_INJECT=launch)", what);
  qsvm::SweepArgs a{};
  a.gen_a = a.gen_b = static_cast<const float4*>(mps);
  a.K = K;
  a.log_k = o.log_k;
  a.Na = a.Nb = N;
  a.ldk = ldk;
  a.row_begin = 0;
  a.row_end = N;
  a.n = n_qubits;
  a.renorm_every = o.renorm_every;
  a.sym = 1;
  a.diag_mode = o.diag_mode;
  int64_t resident = 0;
  hipError_t e = resident_refine_blocks(reps, &resident);
  if (e == hipSuccess)
    e = qsvm::launch_pairs_fp64(a, reps, pairs, pair_count, max_pairs, resident, static_cast<hipStream_t>(stream));
  return hip_status(e, what);
}

qsvm_status qsvm_autotune(int32_t reps, int32_t n_qubits, int64_t N, void* stream, int32_t* best_variant,
                          float* variant_ms, int32_t n_variant_ms) {
  QSVM_TRACE_RANGE("qsvm_autotune");
  const char* what = "qsvm_autotune";
  qsvm_status s = check_shape(N, n_qubits, reps, what);
  if (s != QSVM_OK) return s;
  if (N > 65536) return fail(QSVM_ERR_INVALID_ARG, "%s: N = %lld above the 65536 tuning limit", what, (long long)N);
  if (variant_ms && n_variant_ms < qsvm::kButterflyVariants)
    return fail(QSVM_ERR_SIZE, "%s: variant_ms holds %d < %d entries", what, n_variant_ms, qsvm::kButterflyVariants);
  if (injected_launch_failure()) return fail(QSVM_ERR_HIP, "%s: injected launch failure (QSVM_FAULT_INJECT=launch)", what);
  int32_t best = 0;
  hipError_t e = qsvm::autotune_run(reps, n_qubits, N, static_cast<hipStream_t>(stream), &best, variant_ms);
  if (e != hipSuccess) return hip_status(e, what);
  if (best_variant) *best_variant = best;
  return ok();
}

int32_t qsvm_get_tuned_variant(int32_t reps, int32_t n_qubits, int64_t N) {
  return qsvm::tuned_variant(reps, n_qubits, N);
}

qsvm_status qsvm_autotune_save(void) {
  if (!qsvm::save_tuned_table())
    return fail(QSVM_ERR_INVALID_ARG, "qsvm_autotune_save: cannot write %s", qsvm::tune_cache_path().c_str());
  return ok();
}

const char* qsvm_autotune_cache_path(void) {
  static thread_local std::string path;
  path = qsvm::tune_cache_path();
  return path.c_str();
}

qsvm_status qsvm_set_tuned_variant(int32_t reps, int32_t n_qubits, int64_t N, int32_t variant) {
  const char* what = "qsvm_set_tuned_variant";
  qsvm_status s = check_shape(N, n_qubits, reps, what);
  if (s != QSVM_OK) return s;
  if (variant < 0 || variant >= qsvm::kButterflyVariants)
    return fail(QSVM_ERR_INVALID_ARG, "%s: variant = %d outside [0, %d)", what, variant, qsvm::kButterflyVariants);
  qsvm::set_tuned_variant(reps, n_qubits, N, variant);
  return ok();
}

// ---- state-vector engine ----

size_t qsvm_sv_bytes(int64_t N, int32_t n_qubits) {
  if (n_qubits < 1 || n_qubits > qsvm::kMaxSvQubits || N < 1) return 0;
  if (N > (INT64_MAX / 16) >> n_qubits) return 0;
  return size_t(N << n_qubits) * 16;
}

qsvm_status qsvm_encode_sv(const double* X, int64_t N, int32_t n_qubits, int32_t reps, void* sv, size_t sv_bytes,
                           void* stream) {
  QSVM_TRACE_RANGE("qsvm_encode_sv");
  const char* what = "qsvm_encode_sv";
  if (n_qubits < 1 || n_qubits > qsvm::kMaxSvQubits)
    return fail(QSVM_ERR_UNSUPPORTED, "%s: n_qubits = %d outside [1, 30]", what, n_qubits);
  if (reps < 1 || reps > qsvm::kMaxSvReps) return fail(QSVM_ERR_INVALID_ARG, "%s: reps = %d outside [1, 16]", what, reps);
  const size_t need = qsvm_sv_bytes(N, n_qubits);
  if (need == 0) return fail(QSVM_ERR_INVALID_ARG, "%s: N = %lld invalid or N * 2^n too large", what, (long long)N);
  if (!X) return fail(QSVM_ERR_INVALID_ARG, "%s: X is NULL", what);
  if (!sv) return fail(QSVM_ERR_INVALID_ARG, "%s: sv is NULL", what);
  if (reinterpret_cast<uintptr_t>(sv) % 16 != 0) return fail(QSVM_ERR_INVALID_ARG, "%s: sv is not 16-byte aligned", what);
  if (reinterpret_cast<uintptr_t>(X) % 8 != 0) return fail(QSVM_ERR_INVALID_ARG, "%s: X is not 8-byte aligned", what);
  if (sv_bytes < need) return fail(QSVM_ERR_SIZE, "%s: sv_bytes = %zu < %zu needed", what, sv_bytes, need);
  if (injected_launch_failure()) return fail(QSVM_ERR_HIP, "%s: injected launch failure (QSVM_FAULT_INJECT=launch)", what);
  return hip_status(qsvm::launch_encode_sv(X, N, n_qubits, reps, sv, static_cast<hipStream_t>(stream)), what);
}

namespace {

qsvm_status run_sv_gram(const void* sv_a, int64_t Na, const void* sv_b, int64_t Nb, int32_t n, double* K,
                        int64_t ldk, const qsvm_gram_opts* opts, bool sym, void* stream, const char* what) {
  using qsvm::kTile;
  if (!sv_a || !sv_b) return fail(QSVM_ERR_INVALID_ARG, "%s: state buffer is NULL", what);
  if (!K) return fail(QSVM_ERR_INVALID_ARG, "%s: K is NULL", what);
  if (n < 1 || n > qsvm::kMaxSvQubits) return fail(QSVM_ERR_UNSUPPORTED, "%s: n_qubits = %d outside [1, 30]", what, n);
  if (qsvm_sv_bytes(Na, n) == 0 || qsvm_sv_bytes(Nb, n) == 0 || Na > kMaxN || Nb > kMaxN)
    return fail(QSVM_ERR_INVALID_ARG, "%s: N invalid or N * 2^n too large", what);
  if (ldk < Nb) return fail(QSVM_ERR_INVALID_ARG, "%s: ldk = %lld < %lld", what, (long long)ldk, (long long)Nb);
  if ((reinterpret_cast<uintptr_t>(sv_a) | reinterpret_cast<uintptr_t>(sv_b)) % 16 != 0)
    return fail(QSVM_ERR_INVALID_ARG, "%s: state buffer is not 16-byte aligned", what);
  Opts o;
  qsvm_status s = read_opts(opts, Na, o, what);
  if (s != QSVM_OK) return s;
  if (!sym) o.diag_mode = 0;
  const int64_t tiles_b = (Nb + kTile - 1) / kTile;
  if (tiles_b > qsvm::kMaxGridBlocks)  // one block per tile; one row per launch at least
    return fail(QSVM_ERR_UNSUPPORTED, "%s: Nb = %lld: one row of %lld tiles exceeds one launch", what, (long long)Nb,
                (long long)tiles_b);
  if (o.row_end <= o.row_begin) return ok();
  qsvm::SweepArgs a{};
  a.K = K;
  a.log_k = o.log_k;
  a.Na = Na;
  a.Nb = Nb;
  a.ldk = ldk;
  a.row_begin = o.row_begin;
  a.row_end = o.row_end;
  a.n = n;
  a.sym = sym ? 1 : 0;
  a.diag_mode = o.diag_mode;
  a.tile_row0 = int32_t(o.row_begin / kTile);
  a.tile_rows = int32_t((o.row_end - 1) / kTile) - a.tile_row0 + 1;
  a.tiles_b = int32_t(tiles_b);
  if (injected_launch_failure()) return fail(QSVM_ERR_HIP, "%s: injected launch failure (QSVM_FAULT_INJECT=launch)", what);
  return hip_status(qsvm::launch_sv_gram(a, sv_a, sv_b, n, static_cast<hipStream_t>(stream)), what);
}

}  // namespace

qsvm_status qsvm_sv_gram(const void* sv_a, int64_t Na, const void* sv_b, int64_t Nb, int32_t n_qubits, double* K,
                         int64_t ldk, const qsvm_gram_opts* opts, void* stream) {
  QSVM_TRACE_RANGE("qsvm_sv_gram");
  return run_sv_gram(sv_a, Na, sv_b, Nb, n_qubits, K, ldk, opts, false, stream, "qsvm_sv_gram");
}

qsvm_status qsvm_sv_gram_sym(const void* sv, int64_t N, int32_t n_qubits, double* K, int64_t ldk,
                             const qsvm_gram_opts* opts, void* stream) {
  QSVM_TRACE_RANGE("qsvm_sv_gram_sym");
  return run_sv_gram(sv, N, sv, N, n_qubits, K, ldk, opts, true, stream, "qsvm_sv_gram_sym");
}

const char* qsvm_status_string(qsvm_status s) {
  switch (s) {
    case QSVM_OK: return "QSVM_OK";
    case QSVM_ERR_INVALID_ARG: return "QSVM_ERR_INVALID_ARG: invalid argument";
    case QSVM_ERR_UNSUPPORTED: return "QSVM_ERR_UNSUPPORTED: request outside the supported range";
    case QSVM_ERR_HIP: return "QSVM_ERR_HIP: HIP runtime or launch failure";
    case QSVM_ERR_SIZE: return "QSVM_ERR_SIZE: caller buffer too small";
  }
  return "unknown qsvm_status";
}

const char* qsvm_last_error(void) { return g_last_error.c_str(); }

int32_t qsvm_abi_version(void) { return 2; }

}  // extern "C"
