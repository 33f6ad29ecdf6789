// Launch trace: when enabled, every traced kernel launch is bracketed by a
// pair of HIP events recorded on the stream it is launched on, so the
// elapsed time between them is that kernel's duration on the device.
// Records are aggregated per (label, p, precision) when read.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "fem.h"
#include "fem_internal.h"
#include "trace.h"

namespace fem {
namespace {

struct Span {
    const char* label;
    int p, prec;
    hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Span> g_spans;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

bool trace_on() { return g_on; }

int trace_begin(const char* label, int p, int prec, hipStream_t s) {
    if (!g_on) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t a = take_event(), b = take_event();
    if (!a || !b) return -1;
    if (hipEventRecord(a, s) != hipSuccess) {
        g_pool.push_back(a);
        g_pool.push_back(b);
        return -1;
    }
    g_spans.push_back(Span{label, p, prec, a, b});
    return (int)g_spans.size() - 1;
}

void trace_end(int id, hipStream_t s) {
    if (id < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (id >= (int)g_spans.size()) return;
    hipEventRecord(g_spans[id].b, s);
}

}  // namespace fem

using namespace fem;

extern "C" fem_status fem_trace_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (Span& sp : g_spans) {
        hipEventSynchronize(sp.b);
        g_pool.push_back(sp.a);
        g_pool.push_back(sp.b);
    }
    g_spans.clear();
    g_on = on != 0;
    return FEM_OK;
}

extern "C" int fem_trace_read(fem_trace_rec* out, int max_recs) {
    std::lock_guard<std::mutex> lk(g_mu);
    std::map<std::tuple<std::string, int, int>, std::pair<int, double>> agg;
    for (Span& sp : g_spans) {
        if (hipEventSynchronize(sp.b) != hipSuccess) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, sp.a, sp.b) != hipSuccess) continue;
        auto& v = agg[std::make_tuple(std::string(sp.label), sp.p, sp.prec)];
        v.first += 1;
        v.second += ms;
        g_pool.push_back(sp.a);
        g_pool.push_back(sp.b);
    }
    g_spans.clear();
    int n = 0;
    for (auto& kv : agg) {
        if (out && n < max_recs) {
            fem_trace_rec& r = out[n];
            std::memset(&r, 0, sizeof(r));
            std::strncpy(r.label, std::get<0>(kv.first).c_str(), sizeof(r.label) - 1);
            r.p = std::get<1>(kv.first);
            r.prec = std::get<2>(kv.first);
            r.launches = kv.second.first;
            r.total_ms = kv.second.second;
        }
        ++n;
    }
    return n;
}
