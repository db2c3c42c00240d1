// common.hpp -- host-side pieces shared by the translation units of libsdmm: option and
// pointer bundles passed to kernels, the workspace layout, and launch helpers defined in
// fit.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>

#include "../../include/sdmm.h"
#include "device_math.hpp"

namespace sdmm {

struct DevOpts {
    int K, eta_mode, prior_mode, flags, min_samples, pad;
    double eta, rm_alpha, rm_beta, prior_scale, prior_q, prior_a, prior_b[5], dead_threshold;
};

struct MixPtrs {
    double *pi, *mud, *mux, *cov;
};

struct StatePtrs {
    double *s0, *s2, *sw;
    int32_t* step;
};

// Workspace: FP32 mirrors, per-cell flags, chunk tables and per-chunk FP64 records. The
// record is sized for the larger (adjoint) pass so one workspace serves every call.
struct Layout {
    size_t mirror, flags, chunk_start, chunk_cell, n_total, partial, total;
    int64_t tmax;
    int ps_fit, ps_grad;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline int default_chunk(const sdmm_fit_opts* o) { return o->chunk > 0 ? o->chunk : 1024; }
inline int default_waves(const sdmm_fit_opts* o) { return o->waves > 0 ? o->waves : 4; }

inline Layout layout_for(int32_t C, int32_t K, int64_t N, int64_t chunk)
{
    Layout L{};
    L.tmax = (int64_t)C + (N + chunk - 1) / chunk;
    L.ps_fit = (kStats * K + 3 + 1) & ~1;
    L.ps_grad = ((kStats + 2) * K + 4 + 1) & ~1;
    size_t p = 0;
    L.mirror = p;
    p = align256(p + (size_t)C * K * kMirror * sizeof(float));
    L.flags = p;
    p = align256(p + (size_t)C * sizeof(int32_t));
    L.chunk_start = p;
    p = align256(p + (size_t)(C + 1) * sizeof(int32_t));
    L.chunk_cell = p;
    p = align256(p + (size_t)L.tmax * sizeof(int32_t));
    L.n_total = p;
    p = align256(p + sizeof(int32_t));
    L.partial = p;
    p = align256(p + (size_t)L.tmax * (size_t)L.ps_grad * sizeof(double));
    L.total = p;
    return L;
}

// component lanes per sample: K rounded up to a power of two, at least 4
inline int group_for(int K)
{
    int G = 4;
    while (G < K) G <<= 1;
    return G;
}

inline int check(hipError_t e)
{
    if (e != hipSuccess) {
        fprintf(stderr, "libsdmm: HIP error %s\n", hipGetErrorString(e));
        return SDMM_EDEVICE;
    }
    return SDMM_OK;
}

inline DevOpts dev_opts(const sdmm_fit_opts* o)
{
    DevOpts d{};
    d.K = o->K;
    d.eta_mode = o->eta_mode;
    d.prior_mode = o->prior_mode;
    d.flags = o->flags;
    d.min_samples = o->min_samples;
    d.eta = o->eta;
    d.rm_alpha = o->rm_alpha;
    d.rm_beta = o->rm_beta;
    d.prior_scale = o->prior_scale;
    d.prior_q = o->prior_q;
    d.prior_a = o->prior_a;
    for (int i = 0; i < 5; ++i) d.prior_b[i] = o->prior_b[i];
    d.dead_threshold = o->dead_threshold;
    return d;
}

// common argument checks of the fit and adjoint entry points
int validate_fit_args(const int64_t* cell_offsets, const float* samples, int64_t n_samples,
                      const sdmm_mixtures* mix, const sdmm_fit_opts* opts, const int32_t* cell_status,
                      const void* workspace, size_t workspace_bytes);

// plan (chunk table, cleared status and flags) + FP32 mirrors, enqueued on s
void launch_plan_prepare(const int64_t* off, int64_t N, const sdmm_mixtures& mix, int64_t chunk, int32_t* status,
                         char* ws, const Layout& L, hipStream_t s);

}  // namespace sdmm
