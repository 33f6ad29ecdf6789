// Kernel launch trace (see trace.cpp).  Usage at a launch site:
//     TraceSpan ts("pi_solve", P, prec_of<S>(), s);
//     hipLaunchKernelGGL(...);
// The span ends (its stop event is recorded) when ts leaves scope.
#pragma once
#include <hip/hip_runtime.h>

namespace fem {

bool trace_on();
int trace_begin(const char* label, int p, int prec, hipStream_t s);
void trace_end(int id, hipStream_t s);

struct TraceSpan {
    int id;
    hipStream_t s;
    TraceSpan(const char* label, int p, int prec, hipStream_t st)
        : id(trace_on() ? trace_begin(label, p, prec, st) : -1), s(st) {}
    ~TraceSpan() { trace_end(id, s); }
    TraceSpan(const TraceSpan&) = delete;
    TraceSpan& operator=(const TraceSpan&) = delete;
};

}  // namespace fem
