// qsvm_gram_sym_noalloc: the symmetric Gram for callers that cannot allocate
// device memory (work recorded under stream capture, tight serving loops,
// harnesses that forbid hipMalloc).  The only device memory qsvm_gram_sym
// takes beyond its inputs and outputs is the FP64 refinement's tile list
// ([count, tile indices...], a stream-ordered temporary there); here it lives
// in the file-scope array `scratch`, one copy per device for the life of the
// process.  The sweep and refinement kernels are the same, so results are
// bitwise those of qsvm_gram_sym.

#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/qsvm.h"
#include "qsvm_internal.h"
#include "trace.h"

namespace qsvm {
qsvm_status gram_sym_static_workspace(const void* mps, int64_t N, int32_t n_qubits, int32_t reps, double* K,
                                      int64_t ldk, const qsvm_gram_opts* opts, void* stream,
                                      hipError_t (*get_ws)(uint32_t**), int64_t ws_entries, const char* what);
}

namespace {

// [count, tile list...] of the refinement: one entry for the count and one per
// tile of a launch chunk (4 MiB per device).
constexpr int64_t kScratchEntries = QSVM_NOALLOC_SCRATCH_ENTRIES;

static __device__ __align__(256) uint32_t scratch[kScratchEntries];

constexpr int kMaxDevices = 64;
std::mutex g_setup;
uint32_t* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device (null until set up)

// Device address of this device's `scratch`, looked up once per device with
// that device current.  In host code the array's name is only a host-side
// stand-in, so kernels receive this address, never `scratch` itself.
hipError_t scratch_address(uint32_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_setup);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<uint32_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" qsvm_status qsvm_gram_sym_noalloc(const void* mps, int64_t N, int32_t n_qubits, int32_t reps, double* K,
                                             int64_t ldk, const qsvm_gram_opts* opts, void* stream) {
  QSVM_TRACE_RANGE("qsvm_gram_sym_noalloc");
  return qsvm::gram_sym_static_workspace(mps, N, n_qubits, reps, K, ldk, opts, stream, scratch_address,
                                         kScratchEntries, "qsvm_gram_sym_noalloc");
}
