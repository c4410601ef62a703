// roctx ranges and marks on the host side of the library (rocprofv3
// --marker-trace shows them beside the kernels): a render call, a PSF-FT
// cache fill, a server submission, a batch launch, a batch completion.
// Without a profiler attached each call is a cheap no-op.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace gfc {

// A roctx range for the enclosing scope.
class TraceScope {
 public:
  explicit TraceScope(const char* name) { roctxRangePushA(name); }
  ~TraceScope() { roctxRangePop(); }
  TraceScope(const TraceScope&) = delete;
  TraceScope& operator=(const TraceScope&) = delete;
};

inline void trace_mark(const char* name) { roctxMarkA(name); }

}  // namespace gfc
