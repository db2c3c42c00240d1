// timing.hip -- optional HIP-event timing of the library's kernels by class, recorded on
// the stream each kernel is launched on (eager launches only; graph replays are not
// bracketed). Used by the benchmark to measure kernel durations live.
#include <mutex>
#include <vector>

#include "common.hpp"
#include "timing.hpp"

namespace sdmm {

namespace {
std::mutex g_mu;
bool g_enabled = false;
struct Pair {
    hipEvent_t a, b;
};
std::vector<Pair> g_pairs[kTimerClasses];
}  // namespace

bool timing_enabled() { return g_enabled; }

void timing_begin(int cls, hipStream_t s, void** token)
{
    *token = nullptr;
    if (!g_enabled || cls < 0 || cls >= kTimerClasses) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    Pair* p = new Pair;
    if (hipEventCreate(&p->a) != hipSuccess || hipEventCreate(&p->b) != hipSuccess) {
        delete p;
        return;
    }
    (void)hipEventRecord(p->a, s);
    *token = p;
}

void timing_end(int cls, hipStream_t s, void* token)
{
    if (!token) return;
    Pair* p = static_cast<Pair*>(token);
    (void)hipEventRecord(p->b, s);
    std::lock_guard<std::mutex> lk(g_mu);
    g_pairs[cls].push_back(*p);
    delete p;
}

}  // namespace sdmm

using namespace sdmm;

extern "C" int sdmm_timing_enable(int enable)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_enabled = enable != 0;
    return SDMM_OK;
}

extern "C" int sdmm_timing_read(int kernel_class, double* total_ms, int64_t* launches, int reset)
{
    if (kernel_class < 0 || kernel_class >= kTimerClasses || !total_ms || !launches) return SDMM_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    double tot = 0.0;
    for (const Pair& p : g_pairs[kernel_class]) {
        if (hipEventSynchronize(p.b) != hipSuccess) return SDMM_EDEVICE;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) return SDMM_EDEVICE;
        tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)g_pairs[kernel_class].size();
    if (reset) {
        for (const Pair& p : g_pairs[kernel_class]) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
        g_pairs[kernel_class].clear();
    }
    return SDMM_OK;
}
