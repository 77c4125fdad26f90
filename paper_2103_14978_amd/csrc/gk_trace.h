// Host-side trace ranges of the library's pipeline stages (roctx): each
// entry point, and inside gk_filter_host and the serving loop each stage a
// host thread spends time in, is a named range on the calling thread.
// rocprofv3 --marker-trace records them next to the kernels; without a
// profiler attached a range costs two calls that return at once.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace gkd {

inline void trace_push(const char *name) { roctxRangePushA(name); }
inline void trace_pop() { roctxRangePop(); }

class TraceRange {
  public:
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace gkd
