// Host-side trace ranges (roctx): every entry point that enqueues device work marks its span, and
// the solve marks each SCP iteration it enqueues, so `rocprofv3 --marker-trace` lines the host
// calls up with the kernels they launch.  Without an attached tool the calls do nothing.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace scp {

struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace scp
