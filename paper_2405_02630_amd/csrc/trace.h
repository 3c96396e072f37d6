// Optional roctx ranges around the C-ABI entry points, for timelines taken
// with `rocprofv3 --marker-trace`.  Enabled by QSVM_ROCTX=1 in the
// environment (read once); the marker library (librocprofiler-sdk-roctx) is
// then opened at run time, so the library has no link-time dependency on it.
// A range covers the host side of a call: validation and the enqueueing of
// its kernels (the kernels themselves run asynchronously).
#pragma once

namespace qsvm {

class TraceRange {
 public:
  explicit TraceRange(const char* name);
  ~TraceRange();
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;

 private:
  bool pushed_;
};

// True once the marker library has been opened (QSVM_ROCTX=1 and found).
bool trace_enabled();

}  // namespace qsvm

#define QSVM_TRACE_RANGE(name) ::qsvm::TraceRange qsvm_trace_range_(name)
