// Per-launch kernel timing (see trace.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace stem {

bool trace_enabled();

// Records a start event on construction and a stop event on destruction, on stream s,
// under `name`, while tracing is enabled.
class TraceScope {
 public:
  TraceScope(const char* name, hipStream_t s);
  ~TraceScope();
  TraceScope(const TraceScope&) = delete;
  TraceScope& operator=(const TraceScope&) = delete;

 private:
  hipStream_t stream_;
  hipEvent_t stop_;
};

}  // namespace stem

#define STEM_TRACE_CAT2(a, b) a##b
#define STEM_TRACE_CAT(a, b) STEM_TRACE_CAT2(a, b)
#define STEM_TRACE(name, stream) ::stem::TraceScope STEM_TRACE_CAT(trace_scope_, __LINE__)(name, stream)
