// Named ranges around the library's entry points for tracing tools
// (rocprofv3 --marker-trace shows them beside the kernels they launch).
// Without a tool attached the calls return at once.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace kpd {

struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace kpd
