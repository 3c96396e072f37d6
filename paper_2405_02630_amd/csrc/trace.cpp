// roctx ranges for the C-ABI entry points (see trace.h).

#include "trace.h"

#include <dlfcn.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

namespace qsvm {
namespace {

typedef int (*PushFn)(const char*);
typedef int (*PopFn)(void);

PushFn g_push = nullptr;
PopFn g_pop = nullptr;
std::once_flag g_once;

void open_markers() {
  const char* v = getenv("QSVM_ROCTX");
  if (!v || strcmp(v, "1") != 0) return;
  void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
  if (!h) h = dlopen("librocprofiler-sdk-roctx.so", RTLD_NOW | RTLD_LOCAL);
  if (!h) return;
  PushFn push = reinterpret_cast<PushFn>(dlsym(h, "roctxRangePushA"));
  PopFn pop = reinterpret_cast<PopFn>(dlsym(h, "roctxRangePop"));
  if (push && pop) {
    g_push = push;
    g_pop = pop;
  }
}

}  // namespace

bool trace_enabled() {
  std::call_once(g_once, open_markers);
  return g_push != nullptr;
}

TraceRange::TraceRange(const char* name) : pushed_(false) {
  if (trace_enabled()) {
    g_push(name);
    pushed_ = true;
  }
}

TraceRange::~TraceRange() {
  if (pushed_) g_pop();
}

}  // namespace qsvm
