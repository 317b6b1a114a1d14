// lb_trace.h -- roctx ranges over the library's C-ABI calls (host code), so
// that a profiler's marker trace shows each call around the kernels it
// launches.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace lbnr {

struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePush(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

} // namespace lbnr
