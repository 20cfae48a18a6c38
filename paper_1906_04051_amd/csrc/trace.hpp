// Host-side phase ranges for rocprofv3's marker trace (`--marker-trace`):
// setup, solve, each refinement of a mixed-precision solve, each restart
// cycle (from its enqueue to the host seeing its control block), adjoint,
// batched and block solves, autotuning and value updates.  Enabled when the
// environment variable GMRES_TRACE is set to a value other than "0" (read on
// every API call, so a process can switch it); otherwise no roctx call is
// made.
#pragma once
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdlib>

namespace gm {

inline bool trace_on() {
    const char* v = std::getenv("GMRES_TRACE");
    return v && v[0] && !(v[0] == '0' && v[1] == 0);
}

// Nested range for the lifetime of the object.
struct TraceRange {
    bool on;
    explicit TraceRange(const char* name) : on(trace_on()) {
        if (on) roctxRangePushA(name);
    }
    ~TraceRange() {
        if (on) roctxRangePop();
    }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

// Range that may overlap its neighbours (restart cycles are pipelined: cycle
// c + 1 is enqueued before cycle c is seen to finish).
struct TraceSpan {
    bool on = false;
    roctx_range_id_t id = 0;
    void start(const char* name) {
        on = trace_on();
        if (on) id = roctxRangeStartA(name);
    }
    void stop() {
        if (on) roctxRangeStop(id);
        on = false;
    }
};

}  // namespace gm
