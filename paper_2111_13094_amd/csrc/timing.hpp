// timing.hpp -- hooks of the optional per-kernel-class event timing (timing.hip)
#pragma once

#include <hip/hip_runtime.h>

namespace sdmm {

constexpr int kTimerClasses = 8;  // SDMM_TIMER_* in sdmm.h

bool timing_enabled();
void timing_begin(int cls, hipStream_t s, void** token);
void timing_end(int cls, hipStream_t s, void* token);

// brackets the launches in its scope with events when timing is enabled
struct ScopedTimer {
    int cls;
    hipStream_t s;
    void* token = nullptr;
    ScopedTimer(int c, hipStream_t st) : cls(c), s(st) { timing_begin(cls, s, &token); }
    ~ScopedTimer() { timing_end(cls, s, token); }
};

}  // namespace sdmm
