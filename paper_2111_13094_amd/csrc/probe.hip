// probe.hip -- device microbenchmarks of the vector FMA rates this library's code
// generation reaches on the chip (FP32 without packed instructions, and FP64), so that
// the measured rates of the method's kernels can be set against what the SIMDs issue for
// code built like theirs as well as against the published peaks (which count packed
// FP32). Measurement support only: no step of the method runs here.
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace sdmm {

constexpr int kProbeChains = 16;  // independent FMA chains per thread

// every thread runs `iters` rounds of kProbeChains independent FMAs (a <- a * m + c) and
// stores the chains' sum, so that none of the work is dead
template <typename T>
__global__ __launch_bounds__(256) void fma_probe_kernel(int iters, T m, T c, T* __restrict__ out)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    T a[kProbeChains];
#pragma unroll
    for (int j = 0; j < kProbeChains; ++j) a[j] = (T)(tid & 255) * (T)1e-3 + (T)j;
    // four rounds (64 FMAs) per loop trip, so that loop control is a small share of the issue
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kProbeChains; ++j) a[j] = fma(a[j], m, c);
    }
    T s = 0;
#pragma unroll
    for (int j = 0; j < kProbeChains; ++j) s += a[j];
    out[tid] = s;
}

}  // namespace sdmm

using namespace sdmm;

extern "C" int sdmm_probe_fma(int32_t bits, int32_t n_groups, int32_t iters, void* out, double* ms, void* stream)
{
    if ((bits != 32 && bits != 64) || n_groups < 1 || iters < 1 || !out || !ms) return SDMM_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return SDMM_EDEVICE;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return SDMM_EDEVICE;
    }
    (void)hipEventRecord(a, s);
    if (bits == 32)
        fma_probe_kernel<float><<<n_groups, 256, 0, s>>>(iters, 0.999999f, 1e-6f, static_cast<float*>(out));
    else
        fma_probe_kernel<double><<<n_groups, 256, 0, s>>>(iters, 0.999999999, 1e-9, static_cast<double*>(out));
    int rc = check(hipGetLastError());
    (void)hipEventRecord(b, s);
    float t = 0.0f;
    if (rc == SDMM_OK) rc = check(hipEventSynchronize(b));
    if (rc == SDMM_OK) rc = check(hipEventElapsedTime(&t, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = (double)t;
    return rc;
}
