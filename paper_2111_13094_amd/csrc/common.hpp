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

// Workspace: FP32 mirrors, per-cell flags and arrival counters, the offsets check, and the
// records of the E-step (one per record slot; C + W slots with W = ceil(N / P)), sized
// for FP64 elements (EM passes with FP32 block sums use FP32 elements at the same stride).
// Records are sized for the larger (adjoint) pass so one workspace serves every call.
struct Layout {
    int wpb;  // waves per work group of the E-step launch
    size_t mirror, flags, arrive, global_ok, records, total;  // global_ok: int32[3] control words
    int64_t P;  // samples per E-step work item, 2^ps
    int ps;
    int W;
    int ps_fit, ps_grad;
    int32_t max_cell;  // the caller's bound on samples per cell (0: none)
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// component lanes per sample: K rounded up to a power of two, at least 4
inline int group_for(int K)
{
    int G = 4;
    while (G < K) G <<= 1;
    return G;
}


// E-step work items of 256 samples (about 47 us of one wave at 4 waves per SIMD for
// K = 16): small enough that the launch tail is short, large enough that the per-item
// record (21 G + 3 doubles) and the M-step's read of it stay cheap.
constexpr int kDefaultWaves = 1 << 16;  // cap on the number of items; P grows beyond it
constexpr int kDefaultMinSamplesPerWave = 256;

inline Layout layout_for(int32_t C, int32_t K, int64_t N, const sdmm_fit_opts* o)
{
    Layout L{};
    L.wpb = (o->waves_per_block == 2 || o->waves_per_block == 4) ? o->waves_per_block : 1;
    const int64_t wmax = o->max_ranges > 0 ? o->max_ranges : kDefaultWaves;
    const int64_t pmin = o->min_range > 0 ? o->min_range : kDefaultMinSamplesPerWave;
    int64_t P = (N + wmax - 1) / wmax;
    if (P < pmin) P = pmin;
    L.ps = 0;
    while ((int64_t(1) << L.ps) < P) ++L.ps;  // a power of two: item maps are shifts
    P = int64_t(1) << L.ps;
    L.P = P;
    L.W = N > 0 ? (int)((N + P - 1) / P) : 0;
    L.max_cell = o->max_cell_samples;
    const int G = group_for(K);  // records keep statistic s of component k at s * G + k
    L.ps_fit = (kStats * G + 3 + 1) & ~1;
    L.ps_grad = ((kStats + 2) * G + 4 + 1) & ~1;
    size_t p = 0;
    L.mirror = p;
    p = align256(p + (size_t)C * K * kMirror * sizeof(float));
    L.flags = p;
    p = align256(p + (size_t)C * sizeof(int32_t));
    L.arrive = p;
    p = align256(p + (size_t)C * sizeof(int32_t));
    L.global_ok = p;
    p = align256(p + 3 * sizeof(int32_t));
    L.records = p;
    p = align256(p + ((size_t)C + (size_t)L.W) * (size_t)L.ps_grad * sizeof(double));
    L.total = p;
    return L;
}

// lanes per cell in the M-step and setup kernels: K rounded up to a power of two
inline int group_pow2(int K)
{
    int G = 1;
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

typedef void (*EstepFn)(const float*, int64_t, const int64_t*, int, int, int64_t, int64_t, const float*, int, int,
                        void*, int32_t*, int);

// E-step kernel for G component lanes, running-sum variant, Jacobian option, adjoint pass
EstepFn estep_function(int G, int acc, bool jac, bool adj);
// FP64 adjoint pass for G component lanes
EstepFn adj64_function(int G);

// setup kernel: FP32 mirrors (full: with the adjoint's twist rates and residues),
// status reset, per-cell flags and the offsets check
void launch_setup(const int64_t* off, int64_t N, const sdmm_mixtures& mix, int32_t* status, char* ws,
                  const Layout& L, hipStream_t s, bool full);

// record tree levels after an E-step pass (all cells, or one cell when cell >= 0, whose
// samples are [c0, c1)); the pass names the record layout, rec32 the FP32 element type
// of EM records (adjoint records are FP64)
enum TreePass { kTreeFit = 0, kTreeGrad = 1 };
void launch_tree(TreePass pass, const int64_t* off, int64_t N, int C, int K, const Layout& L, int cell, int64_t c0,
                 int64_t c1, char* ws, hipStream_t s, bool rec32);

// stepwise EM of every cell (one wave per cell), after launch_setup
void launch_stepwise(const int64_t* off, const float* smp, int64_t N, const sdmm_mixtures& mix,
                     const sdmm_em_state& st, const sdmm_fit_opts& opts, int32_t* status, const Layout& L, char* ws,
                     hipStream_t s);

// E-step over the items in record slots [slot_lo, slot_hi), one wave per slot; with
// check, one more work group writes the offsets-check control words (the setup kernel's
// job when it runs)
void launch_estep(EstepFn est, const float* smp, int64_t N, const int64_t* off, int C, int K, const Layout& L,
                  int64_t slot_lo, int64_t slot_hi, int PS, char* ws, hipStream_t s, bool check = false);

// Host-side record of which workspace holds E-step mirrors of the current parameters of
// which mixture arrays: a batched fit with SDMM_FLAG_CARRY_MIRRORS writes them in its
// last M-step and marks the workspace; any other use of the workspace clears the mark.
bool mirrors_carried(const void* ws, const sdmm_mixtures& mix);
void mark_mirrors(const void* ws, const sdmm_mixtures& mix, bool carried);

}  // namespace sdmm
