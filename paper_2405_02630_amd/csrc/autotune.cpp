// Autotuner for the butterfly sweep: times every kernel variant (ket points
// per lane x register budget) on a synthetic symmetric Gram of the requested
// shape and records the fastest in a table keyed by (GPU architecture, reps,
// floor(log2 n), floor(log2 N)) -- the best variant depends on the chain
// length and on how many tiles there are to fill the device with.  The table
// is persisted in a small text cache file, read once per architecture on
// first use, so later processes start tuned; Gram calls with
// opts.variant == 0 and batch plans consult it.

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/qsvm.h"
#include "qsvm_internal.h"
#include "sweep_common.h"

namespace qsvm {
namespace {

constexpr int kBuckets = 17;   // n-bucket = floor(log2 n), n <= 65535
constexpr int kNBuckets = 40;  // N-bucket = floor(log2 N)
using Key = std::tuple<std::string, int, int, int>;  // (arch, reps, n-bucket, N-bucket)

std::mutex g_mu;
std::map<Key, int> g_table;           // tuned variants
std::set<std::string> g_loaded_arch;  // architectures whose cache entries are loaded
std::string g_arch[64];               // architecture name per device id ("" = not looked up)

int bucket_of(int64_t v, int buckets) {
  int b = 0;
  while ((int64_t(1) << (b + 1)) <= v && b + 1 < buckets) ++b;
  return b;
}

// Cache file: $QSVM_TUNE_CACHE if set (empty = no persistence), else
// $XDG_CACHE_HOME/qsvm/autotune.txt or $HOME/.cache/qsvm/autotune.txt.
std::string cache_path() {
  const char* p = getenv("QSVM_TUNE_CACHE");
  if (p) return std::string(p);
  const char* x = getenv("XDG_CACHE_HOME");
  if (x && *x) return std::string(x) + "/qsvm/autotune.txt";
  const char* h = getenv("HOME");
  if (h && *h) return std::string(h) + "/.cache/qsvm/autotune.txt";
  return std::string();
}

// Architecture of the current device, e.g. "gfx950" (the part of the
// gcnArchName before its feature flags); "unknown" without a device.
std::string current_arch_locked() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return "unknown";
  if (g_arch[dev].empty()) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a(prop.gcnArchName);
    const size_t c = a.find(':');
    g_arch[dev] = (c == std::string::npos) ? a : a.substr(0, c);
    if (g_arch[dev].empty()) g_arch[dev] = "unknown";
  }
  return g_arch[dev];
}

// One cache line: "<arch> <reps> <n-bucket> <N-bucket> <variant>"; '#' starts
// a comment; malformed lines are ignored.
bool parse_line(const char* line, Key& k, int& variant) {
  char a[64];
  int reps, nb, Nb;
  if (line[0] == '#') return false;
  if (sscanf(line, "%63s %d %d %d %d", a, &reps, &nb, &Nb, &variant) != 5) return false;
  if (reps < 1 || reps > kMaxReps || nb < 0 || nb >= kBuckets || Nb < 0 || Nb >= kNBuckets || variant < 0 ||
      variant >= kButterflyVariants)
    return false;
  k = Key(a, reps, nb, Nb);
  return true;
}

void load_arch_locked(const std::string& arch) {
  if (g_loaded_arch.count(arch)) return;
  g_loaded_arch.insert(arch);
  const std::string path = cache_path();
  if (path.empty()) return;
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return;
  char line[256];
  while (fgets(line, sizeof line, f)) {
    Key k;
    int v;
    if (parse_line(line, k, v) && std::get<0>(k) == arch && !g_table.count(k)) g_table[k] = v;  // this process's entries win
  }
  fclose(f);
}

// Merge this process's entries into the cache file (entries of other
// architectures and buckets are kept); written to a temporary, then renamed.
bool save_locked() {
  const std::string path = cache_path();
  if (path.empty()) return true;
  std::map<Key, int> merged;
  if (FILE* f = fopen(path.c_str(), "r")) {
    char line[256];
    while (fgets(line, sizeof line, f)) {
      Key k;
      int v;
      if (parse_line(line, k, v)) merged[k] = v;
    }
    fclose(f);
  }
  for (const auto& kv : g_table) merged[kv.first] = kv.second;
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0) {
    // create the directory chain (mkdir -p)
    std::string dir = path.substr(0, slash);
    for (size_t i = 1; i <= dir.size(); ++i)
      if (i == dir.size() || dir[i] == '/') {
        const std::string part = dir.substr(0, i);
        (void)mkdir(part.c_str(), 0755);  // existing directories fail harmlessly
      }
  }
  const std::string tmp = path + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  fprintf(f, "# qsvm butterfly-sweep autotune cache: arch reps floor(log2 n_qubits) floor(log2 N) variant\n");
  for (const auto& kv : merged)
    fprintf(f, "%s %d %d %d %d\n", std::get<0>(kv.first).c_str(), std::get<1>(kv.first), std::get<2>(kv.first),
            std::get<3>(kv.first), kv.second);
  const bool ok = fclose(f) == 0;
  return ok && rename(tmp.c_str(), path.c_str()) == 0;
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

int32_t tuned_variant(int32_t reps, int32_t n, int64_t N) {
  if (reps < 1 || reps > kMaxReps || n < 1 || N < 1) return 0;
  std::lock_guard<std::mutex> lk(g_mu);
  const std::string arch = current_arch_locked();
  load_arch_locked(arch);
  // the entry of this (n, N) bucket, else the built-in default 0: a variant
  // tuned for another point count is not carried over (the best one changes
  // with the number of tiles: 8 waves per SIMD win below ~2048 points at
  // r = 2 and lose 8 % at 4096)
  const auto it = g_table.find(Key(arch, reps, bucket_of(n, kBuckets), bucket_of(N, kNBuckets)));
  return it == g_table.end() ? 0 : it->second;
}

void set_tuned_variant(int32_t reps, int32_t n, int64_t N, int32_t variant) {
  std::lock_guard<std::mutex> lk(g_mu);
  const std::string arch = current_arch_locked();
  load_arch_locked(arch);
  g_table[Key(arch, reps, bucket_of(n, kBuckets), bucket_of(N, kNBuckets))] = variant;
}

bool save_tuned_table() {
  std::lock_guard<std::mutex> lk(g_mu);
  return save_locked();
}

std::string tune_cache_path() { return cache_path(); }

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
    a.gen_a = a.gen_b = static_cast<const float4*>(mps);  // butterfly sweep: no dense tensors
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
  set_tuned_variant(reps, n, N, best_v);
  (void)save_tuned_table();
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
