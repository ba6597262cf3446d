// Event-based kernel and phase timing.  When enabled, a scope records a HIP event
// on its stream at entry and exit; elapsed times are summed when queried.
#include "internal.h"
#include "../../include/adc3ea.h"
#include <atomic>
#include <mutex>
#include <vector>

namespace adc3 {
namespace {
struct Rec {
    hipEvent_t a, b;
    int k;
    double flops, bytes, bound_ms;
};
std::mutex mu;
std::atomic<bool> enabled{false};
std::vector<Rec> recs;
struct Acc {
    double ms = 0, flops = 0, bytes = 0, bound_ms = 0;
    long long n = 0;
} acc[PROF_N];

void drain() {
    for (auto& r : recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            acc[r.k].ms += ms;
            acc[r.k].n += 1;
            acc[r.k].flops += r.flops;
            acc[r.k].bytes += r.bytes;
            acc[r.k].bound_ms += r.bound_ms;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    recs.clear();
}
}  // namespace

ProfScope::ProfScope(int kernel, hipStream_t stream, double f, double b, double bound)
    : k(kernel), s(stream), flops(f), bytes(b), bound_ms(bound) {
    if (!enabled || g_dry) return;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    if (hipEventRecord(e, s) != hipSuccess) { (void)hipEventDestroy(e); return; }
    ev0 = e;
}

ProfScope::~ProfScope() {
    if (!ev0) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    if (hipEventRecord(e, s) != hipSuccess) { (void)hipEventDestroy(e); return; }
    std::lock_guard<std::mutex> g(mu);
    recs.push_back(Rec{(hipEvent_t)ev0, e, k, flops, bytes, bound_ms});
    if (recs.size() > 4096) drain();
}

}  // namespace adc3

extern "C" void adc3_profile_enable(int on) {
    using namespace adc3;
    std::lock_guard<std::mutex> g(mu);
    drain();
    for (auto& a : acc) a = Acc{};
    enabled = on != 0;
}

extern "C" int adc3_profile_query(int kernel, double* total_ms, long long* count, double* flops, double* bytes) {
    using namespace adc3;
    if (kernel < 0 || kernel >= PROF_N) {
        set_error("adc3_profile_query: unknown kernel id");
        return ADC3_EINVAL;
    }
    std::lock_guard<std::mutex> g(mu);
    drain();
    if (total_ms) *total_ms = acc[kernel].ms;
    if (count) *count = acc[kernel].n;
    if (flops) *flops = acc[kernel].flops;
    if (bytes) *bytes = acc[kernel].bytes;
    return ADC3_OK;
}

extern "C" int adc3_profile_query_bound(int kernel, double* bound_ms) {
    using namespace adc3;
    if (kernel < 0 || kernel >= PROF_N || !bound_ms) {
        set_error("adc3_profile_query_bound: unknown kernel id or NULL output");
        return ADC3_EINVAL;
    }
    std::lock_guard<std::mutex> g(mu);
    drain();
    *bound_ms = acc[kernel].bound_ms;
    return ADC3_OK;
}
