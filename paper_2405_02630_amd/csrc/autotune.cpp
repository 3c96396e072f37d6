// Autotuner for the butterfly sweep: times every kernel variant (ket points
// per lane x register budget) on a synthetic symmetric Gram of the requested
// shape and records the fastest in a per-process table, keyed by
// (reps, bucket of n), that launches with opts.variant == 0 consult.

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <mutex>

#include "../../include/qsvm.h"
#include "qsvm_internal.h"
#include "sweep_common.h"

namespace qsvm {
namespace {

constexpr int kBuckets = 17;  // n-bucket = floor(log2 n), n <= 65535
std::mutex g_table_mu;
int8_t g_table[kMaxReps + 1][kBuckets];  // -1 = not tuned
bool g_table_init = false;

int bucket_of(int32_t n) {
  int b = 0;
  while ((1 << (b + 1)) <= n && b + 1 < kBuckets) ++b;
  return b;
}

void ensure_init() {
  if (!g_table_init) {
    memset(g_table, -1, sizeof g_table);
    g_table_init = true;
  }
}

// Deterministic synthetic features in [0, pi): a 64-bit mix of the index.
__global__ void synth_features(double* X, int64_t count, uint64_t seed) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= count) return;
  uint64_t z = uint64_t(t) + seed * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  X[t] = double(z >> 11) * (3.14159265358979323846 / 9007199254740992.0);
}

}  // namespace

int32_t tuned_variant(int32_t reps, int32_t n) {
  std::lock_guard<std::mutex> lk(g_table_mu);
  ensure_init();
  if (reps < 1 || reps > kMaxReps || n < 1) return 0;
  const int v = g_table[reps][bucket_of(n)];
  return v < 0 ? 0 : v;
}

void set_tuned_variant(int32_t reps, int32_t n, int32_t variant) {
  std::lock_guard<std::mutex> lk(g_table_mu);
  ensure_init();
  g_table[reps][bucket_of(n)] = int8_t(variant);
}

hipError_t autotune_run(int32_t reps, int32_t n, int64_t N, hipStream_t stream, int32_t* best,
                        float* ms_out) {
  const int64_t mps_bytes = mps_total_bytes(N, n, reps);
  double* X = nullptr;
  void* mps = nullptr;
  double* K = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipSuccess;
  float best_ms = INFINITY;
  int32_t best_v = 0;
#define QSVM_TRY(x)                 \
  do {                              \
    err = (x);                      \
    if (err != hipSuccess) goto out; \
  } while (0)
  QSVM_TRY(hipMalloc(&X, sizeof(double) * N * n));
  QSVM_TRY(hipMalloc(&mps, mps_bytes));
  QSVM_TRY(hipMalloc(&K, sizeof(double) * N * N));
  QSVM_TRY(hipEventCreate(&e0));
  QSVM_TRY(hipEventCreate(&e1));
  hipLaunchKernelGGL(synth_features, dim3(unsigned((N * n + 255) / 256)), dim3(256), 0, stream, X, N * n,
                     uint64_t(reps * 1000003 + n));
  QSVM_TRY(hipGetLastError());
  QSVM_TRY(launch_encode(X, N, n, reps, mps, stream));
  {
    SweepArgs a{};
    a.gen_a = a.gen_b = reinterpret_cast<const float4*>(static_cast<char*>(mps) + dense_bytes(N, n, reps));
    a.dense_a = a.dense_b = static_cast<const float2*>(mps);
    a.K = K;
    a.Na = a.Nb = N;
    a.ldk = N;
    a.row_begin = 0;
    a.row_end = N;
    a.n = n;
    a.renorm_every = kDefaultRenorm;
    a.sym = 1;
    a.tile_row0 = 0;
    a.tiles_b = a.tile_rows = int32_t((N + kTile - 1) / kTile);
    for (int32_t v = 0; v < kButterflyVariants; ++v) {
      QSVM_TRY(launch_sweep_fast(a, reps, v, stream));  // warm-up
      QSVM_TRY(hipEventRecord(e0, stream));
      for (int r = 0; r < 3; ++r) QSVM_TRY(launch_sweep_fast(a, reps, v, stream));
      QSVM_TRY(hipEventRecord(e1, stream));
      QSVM_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      QSVM_TRY(hipEventElapsedTime(&ms, e0, e1));
      ms /= 3.0f;
      if (ms_out) ms_out[v] = ms;
      if (ms < best_ms) {
        best_ms = ms;
        best_v = v;
      }
    }
  }
  set_tuned_variant(reps, n, best_v);
  if (best) *best = best_v;
out:
#undef QSVM_TRY
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (K) (void)hipFree(K);
  if (mps) (void)hipFree(mps);
  if (X) (void)hipFree(X);
  return err;
}

}  // namespace qsvm
