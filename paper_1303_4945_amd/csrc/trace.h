// Named ranges around the library's entry points for ROCm's tracing tools
// (rocprofv3 --marker-trace records them beside the kernels they enqueue);
// without a tool attached a range costs two calls that return at once.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace sht {

class TraceRange {
public:
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace sht
