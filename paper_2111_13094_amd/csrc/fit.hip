// fit.hip -- batched weighted MAP EM for spatio-directional Gaussian mixtures on gfx950.
//
// Method (Dodik et al., arXiv 2111.13094): statistics of Sec. 3.2 with tangent-space
// coordinates (Sec. 3.1), exp-map mean update and first-order covariance transfer
// (Sec. 3.2, 3.4), Robbins-Monro averaging and MAP updates (Sec. 4.3), one independent
// mixture per spatial cell updated only with at least min_samples vertices (Sec. 4.2).
//
// Kernels per call:            plan (chunk table, status reset) -> prepare (FP32 mirrors)
// per iteration (batched):     estep (all chunks of all cells) -> mstep (all cells)
// per iteration (fused):       estep_fused (last chunk of a cell runs its M-step)
//
// E-step lane mapping: a wave holds 64/G sample slots x G component lanes (G = K rounded
// up to a power of two); each lane evaluates one (sample, component) pair per step, the
// log-sum-exp over components is a DPP all-reduce inside the G-lane group, and each lane
// keeps its component's 21 running sums (FP32 block sums folded into a TwoSum pair).
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "estep.hpp"
#include "timing.hpp"

namespace sdmm {

// ---------------------------------------------------------------------------------
// plan: per-cell chunk counts, exclusive scan, chunk -> cell table; clears status/flags
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void plan_kernel(const int64_t* __restrict__ off, int C, int64_t N,
                                                    int64_t chunk, int32_t* __restrict__ chunk_start,
                                                    int32_t* __restrict__ chunk_cell,
                                                    int32_t* __restrict__ n_total,
                                                    int32_t* __restrict__ status,
                                                    int32_t* __restrict__ flags)
{
    __shared__ int32_t sums[1024];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int per = (C + nt - 1) / nt;
    const int cb = min(C, tid * per), ce = min(C, cb + per);
    int32_t local = 0;
    for (int c = cb; c < ce; ++c) {
        int64_t c0, c1;
        const bool ok = cell_range(off, c, N, c0, c1);
        local += (int32_t)chunks_for(c1 - c0, chunk);
        status[c] = 0;
        flags[c] = ok ? 0 : kFlagBadRange;
    }
    sums[tid] = local;
    __syncthreads();
    for (int d = 1; d < nt; d <<= 1) {
        const int32_t v = tid >= d ? sums[tid - d] : 0;
        __syncthreads();
        sums[tid] += v;
        __syncthreads();
    }
    int32_t base = sums[tid] - local;
    for (int c = cb; c < ce; ++c) {
        chunk_start[c] = base;
        int64_t c0, c1;
        cell_range(off, c, N, c0, c1);
        const int32_t n = (int32_t)chunks_for(c1 - c0, chunk);
        for (int32_t j = 0; j < n; ++j) chunk_cell[base + j] = c;
        base += n;
    }
    if (tid == nt - 1) {
        chunk_start[C] = sums[nt - 1];
        *n_total = sums[nt - 1];
    }
}

__global__ void prepare_kernel(int C, int K, const double* __restrict__ pi, const double* __restrict__ mud,
                               const double* __restrict__ mux, const double* __restrict__ cov,
                               float* __restrict__ mirror, int32_t* __restrict__ flags)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)C * K) return;
    const bool ok = write_mirror(pi[g], mud + 3 * g, mux + 3 * g, cov + 15 * g, mirror + g * kMirror);
    if (!ok) atomicOr(&flags[g / K], kBadParams);
}

template <int G, int ACC, bool JAC>
__global__ __launch_bounds__(256) void estep_kernel(const float* __restrict__ smp, int64_t N,
                                                    const int64_t* __restrict__ off,
                                                    const int32_t* __restrict__ chunk_cell,
                                                    const int32_t* __restrict__ chunk_start,
                                                    const int32_t* __restrict__ n_total,
                                                    const float* __restrict__ mirror, int K,
                                                    int64_t chunk, int chunk_lo, int PS,
                                                    double* __restrict__ partial)
{
    extern __shared__ double lds[];
    const int t = chunk_lo + blockIdx.x;
    if (t >= *n_total) return;
    const int c = chunk_cell[t];
    int64_t c0, c1;
    cell_range(off, c, N, c0, c1);
    const int64_t cs = chunk_size_for(c1 - c0, chunk);
    const int64_t s0 = min(c1, c0 + (int64_t)(t - chunk_start[c]) * cs);
    const int64_t s1 = min(c1, s0 + cs);
    estep_chunk<G, ACC, JAC, false>(smp, N, s0, s1, mirror + (int64_t)c * K * kMirror, K,
                             partial + (int64_t)t * PS, lds);
}

// ---------------------------------------------------------------------------------
// M-step of one cell: reduce its chunk partials (fixed order), gate, Robbins-Monro
// blend and MAP update per component (lane k), new FP32 mirror. One wave per cell.
// ---------------------------------------------------------------------------------
__device__ void mstep_cell(int c, const int32_t* __restrict__ chunk_start, const double* __restrict__ partial,
                           int PS, const int32_t* __restrict__ flags, MixPtrs mix, StatePtrs st,
                           const DevOpts& o, float* __restrict__ mirror, int32_t* __restrict__ status,
                           double* red)
{
    const int K = o.K;
    const int lane = threadIdx.x & 63;
    const int t0 = chunk_start[c], t1 = chunk_start[c + 1];
    const int nv = kStats * K + 3;
    for (int v = lane; v < nv; v += 64) {
        double s = 0.0;
        for (int t = t0; t < t1; ++t) s += partial[(int64_t)t * PS + v];
        red[v] = s;
    }
    __syncthreads();
    const double W = red[kStats * K], Mc = red[kStats * K + 1], negs = red[kStats * K + 2];
    bool fin = isfinite(W);
    for (int v = lane; v < kStats * K; v += 64) fin = fin && isfinite(red[v]);
    fin = __all(fin);
    int gate = 0;
    if (negs > 0.0 || !fin || (flags[c] & kFlagBadRange)) gate = kBadInput;
    else if (flags[c] & kBadParams) gate = kBadParams;
    else if (Mc < (double)o.min_samples) gate = kSkippedFew;
    else if (!(W > 0.0)) gate = kSkippedZeroW;
    if (gate) {
        if (lane == 0) status[c] |= gate;
        return;
    }

    const int j = st.step[c];
    const double eta = j == 0 ? 1.0 : (o.eta_mode == 0 ? o.eta : pow(o.rm_beta * j + 1.0, -o.rm_alpha));
    const double beta = o.prior_mode == 0 ? eta / Mc : o.prior_scale;
    const double hW = j == 0 ? W : (1.0 - eta) * st.sw[c] + eta * W;

    const int k = lane;
    const bool act = k < K;
    const int64_t g = (int64_t)c * K + (act ? k : 0);
    double hS0 = 0.0, hS1[5], hS2[15];
    if (act) {
        hS0 = j == 0 ? red[k] : (1.0 - eta) * st.s0[g] + eta * red[k];
        for (int d = 0; d < 5; ++d) hS1[d] = (j == 0 ? 1.0 : eta) * red[(1 + d) * K + k];
        for (int q = 0; q < 15; ++q)
            hS2[q] = j == 0 ? red[(6 + q) * K + k] : (1.0 - eta) * st.s2[g * 15 + q] + eta * red[(6 + q) * K + k];
    }
    const double bar0 = hS0 / hW;
    double sum0 = act ? bar0 : 0.0;
    for (int ofs = 1; ofs < 64; ofs <<= 1) sum0 += __shfl_xor(sum0, ofs);

    bool dead = false, cholfail = false;
    if (act) {
        double mu[3] = {mix.mud[3 * g], mix.mud[3 * g + 1], mix.mud[3 * g + 2]};
        if (!(bar0 > o.dead_threshold)) {
            dead = true;
            st.s0[g] = hS0;
            for (int q = 0; q < 15; ++q) st.s2[g * 15 + q] = hS2[q];
        } else {
            double m[5];
            for (int d = 0; d < 5; ++d) m[d] = hS1[d] / hS0;
            double Ro[9], Rn[9], mun[3];
            frame64(mu, Ro);
            exp_map64(Ro, m[0], m[1], mun);
            const double nn = sqrt(mun[0] * mun[0] + mun[1] * mun[1] + mun[2] * mun[2]);
            for (int i = 0; i < 3; ++i) mun[i] /= nn;
            frame64(mun, Rn);
            double J[4];
            transfer_jac64(Ro, Rn, m[0], m[1], J);
            // scatter about the new mean in the old frame, then T C T^T with T = blkdiag(J, I3)
            double Cm[5][5];
            for (int d = 0; d < 5; ++d)
                for (int e = 0; e <= d; ++e) {
                    const double v = hS2[tri(d, e)] - hS1[d] * hS1[e] / hS0;
                    Cm[d][e] = v;
                    Cm[e][d] = v;
                }
            double Cn[5][5];
            for (int a = 0; a < 5; ++a)
                for (int b = 0; b < 5; ++b) Cn[a][b] = Cm[a][b];
            for (int b = 0; b < 5; ++b) {  // rows 0,1: J * C
                const double r0 = J[0] * Cm[0][b] + J[1] * Cm[1][b];
                const double r1 = J[2] * Cm[0][b] + J[3] * Cm[1][b];
                Cn[0][b] = r0;
                Cn[1][b] = r1;
            }
            double Tt[5][5];
            for (int a = 0; a < 5; ++a) {  // columns 0,1: (J C) J^T
                Tt[a][0] = Cn[a][0] * J[0] + Cn[a][1] * J[1];
                Tt[a][1] = Cn[a][0] * J[2] + Cn[a][1] * J[3];
                for (int b = 2; b < 5; ++b) Tt[a][b] = Cn[a][b];
            }
            double Sig[15], Lt[15];
            const double den = beta * o.prior_a + bar0;
            for (int d = 0; d < 5; ++d)
                for (int e = 0; e <= d; ++e) {
                    double v = 0.5 * (Tt[d][e] + Tt[e][d]) / hW;
                    if (d == e) v += beta * o.prior_b[d];
                    Sig[tri(d, e)] = v / den;
                }
            for (int i = 0; i < 3; ++i) {
                mix.mud[3 * g + i] = mun[i];
                mix.mux[3 * g + i] += m[2 + i];
            }
            if (chol64<5>(Sig, Lt)) {
                for (int q = 0; q < 15; ++q) mix.cov[g * 15 + q] = Sig[q];
            } else {
                cholfail = true;
            }
            st.s0[g] = hS0;
            for (int d = 0; d < 5; ++d)
                for (int e = 0; e <= d; ++e) st.s2[g * 15 + tri(d, e)] = 0.5 * (Tt[d][e] + Tt[e][d]);
        }
        const double pinew = (beta * o.prior_q + bar0) / ((double)K * beta * o.prior_q + sum0);
        mix.pi[g] = pinew;
        write_mirror(pinew, mix.mud + 3 * g, mix.mux + 3 * g, mix.cov + 15 * g, mirror + g * kMirror);
    }
    const bool any_dead = __any(dead), any_chol = __any(cholfail);
    if (lane == 0) {
        st.sw[c] = hW;
        st.step[c] = j + 1;
        status[c] |= (any_dead ? kDeadComponent : 0) | (any_chol ? kCholFailKeptPrev : 0);
    }
}

__global__ __launch_bounds__(64) void mstep_kernel(const int32_t* __restrict__ chunk_start,
                                                   const double* __restrict__ partial, int PS,
                                                   const int32_t* __restrict__ flags, MixPtrs mix,
                                                   StatePtrs st, DevOpts o, float* __restrict__ mirror,
                                                   int32_t* __restrict__ status, int cell_lo)
{
    __shared__ double red[kStats * kMaxK + 4];
    mstep_cell(cell_lo + blockIdx.x, chunk_start, partial, PS, flags, mix, st, o, mirror, status, red);
}

// ---------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------
typedef void (*EstepFn)(const float*, int64_t, const int64_t*, const int32_t*, const int32_t*, const int32_t*,
                        const float*, int, int64_t, int, int, double*);

template <int G>
static EstepFn estep_for_g(int acc, bool jac)
{
    if (jac) {
        if (acc == kAccPlain) return estep_kernel<G, kAccPlain, true>;
        if (acc == kAccFp64) return estep_kernel<G, kAccFp64, true>;
        return estep_kernel<G, kAccTwoSum, true>;
    }
    if (acc == kAccPlain) return estep_kernel<G, kAccPlain, false>;
    if (acc == kAccFp64) return estep_kernel<G, kAccFp64, false>;
    return estep_kernel<G, kAccTwoSum, false>;
}

static EstepFn estep_for(int G, int acc, bool jac)
{
    switch (G) {
        case 4: return estep_for_g<4>(acc, jac);
        case 8: return estep_for_g<8>(acc, jac);
        case 16: return estep_for_g<16>(acc, jac);
        case 32: return estep_for_g<32>(acc, jac);
        case 64: return estep_for_g<64>(acc, jac);
    }
    return nullptr;
}

struct FitArgs {
    const int64_t* off;
    const float* smp;
    int64_t N;
    sdmm_mixtures mix;
    sdmm_em_state st;
    sdmm_fit_opts opts;
    int32_t* status;
    char* ws;
};

void launch_plan_prepare(const int64_t* off, int64_t N, const sdmm_mixtures& mix, int64_t chunk, int32_t* status,
                         char* ws, const Layout& L, hipStream_t s)
{
    const int C = mix.n_cells, K = mix.K;
    float* mirror = reinterpret_cast<float*>(ws + L.mirror);
    int32_t* flags = reinterpret_cast<int32_t*>(ws + L.flags);
    plan_kernel<<<1, 1024, 0, s>>>(off, C, N, chunk, reinterpret_cast<int32_t*>(ws + L.chunk_start),
                                   reinterpret_cast<int32_t*>(ws + L.chunk_cell),
                                   reinterpret_cast<int32_t*>(ws + L.n_total), status, flags);
    const int64_t nk = (int64_t)C * K;
    prepare_kernel<<<(unsigned)((nk + 255) / 256), 256, 0, s>>>(C, K, mix.weights, mix.mean_dir, mix.mean_pos,
                                                                 mix.cov, mirror, flags);
}

static int enqueue_fit(const FitArgs& a, hipStream_t s, const std::vector<int64_t>* host_off)
{
    const int C = a.mix.n_cells, K = a.opts.K;
    const int64_t chunk = default_chunk(&a.opts);
    const int waves = default_waves(&a.opts);
    const Layout L = layout_for(C, K, a.N, chunk);
    float* mirror = reinterpret_cast<float*>(a.ws + L.mirror);
    int32_t* flags = reinterpret_cast<int32_t*>(a.ws + L.flags);
    int32_t* cstart = reinterpret_cast<int32_t*>(a.ws + L.chunk_start);
    int32_t* ccell = reinterpret_cast<int32_t*>(a.ws + L.chunk_cell);
    int32_t* ntot = reinterpret_cast<int32_t*>(a.ws + L.n_total);
    double* partial = reinterpret_cast<double*>(a.ws + L.partial);
    const MixPtrs mp{a.mix.weights, a.mix.mean_dir, a.mix.mean_pos, a.mix.cov};
    const StatePtrs sp{a.st.s0, a.st.s2, a.st.sw, a.st.step};
    const DevOpts dopt = dev_opts(&a.opts);
    const int G = group_for(K);
    const int acc = (a.opts.flags & SDMM_FLAG_PLAIN_FP32) ? kAccPlain
                    : (a.opts.flags & SDMM_FLAG_FP64_SUMS) ? kAccFp64 : kAccTwoSum;
    const bool jac = (a.opts.flags & SDMM_FLAG_ESTEP_JACOBIAN) != 0;
    EstepFn est = estep_for(G, acc, jac);
    const size_t lds = (size_t)waves * ChunkLayout<false>::kNRed * G * sizeof(double);
    const int ps = L.ps_fit;

    launch_plan_prepare(a.off, a.N, a.mix, chunk, a.status, a.ws, L, s);
    for (int it = 0; it < a.opts.iters; ++it) {
        if (a.opts.schedule == SDMM_SCHED_PER_CELL) {
            int64_t t = 0;
            for (int c = 0; c < C; ++c) {
                const int64_t nch = chunks_for((*host_off)[c + 1] - (*host_off)[c], chunk);
                hipLaunchKernelGGL(est, dim3((unsigned)nch), dim3(waves * 64), lds, s, a.smp, a.N, a.off, ccell,
                                   cstart, ntot, mirror, K, chunk, (int)t, ps, partial);
                mstep_kernel<<<1, 64, 0, s>>>(cstart, partial, ps, flags, mp, sp, dopt, mirror, a.status, c);
                t += nch;
            }
        } else {
            {
                ScopedTimer tm(SDMM_TIMER_ESTEP, s);
                hipLaunchKernelGGL(est, dim3((unsigned)L.tmax), dim3(waves * 64), lds, s, a.smp, a.N, a.off, ccell,
                                   cstart, ntot, mirror, K, chunk, 0, ps, partial);
            }
            ScopedTimer tm(SDMM_TIMER_MSTEP, s);
            mstep_kernel<<<C, 64, 0, s>>>(cstart, partial, ps, flags, mp, sp, dopt, mirror, a.status, 0);
        }
    }
    return check(hipGetLastError());
}

int validate_fit_args(const int64_t* cell_offsets, const float* samples, int64_t n_samples,
                      const sdmm_mixtures* mix, const sdmm_fit_opts* opts, const int32_t* cell_status,
                      const void* workspace, size_t workspace_bytes)
{
    if (!cell_offsets || !mix || !opts || !cell_status || !workspace) return SDMM_EINVAL;
    if (n_samples < 0 || (n_samples > 0 && !samples)) return SDMM_EINVAL;
    if (mix->n_cells <= 0 || mix->K != opts->K || opts->K < 1 || opts->K > kMaxK) return SDMM_EINVAL;
    if (opts->iters < 1 || opts->min_samples < 0) return SDMM_EINVAL;
    if (!mix->weights || !mix->mean_dir || !mix->mean_pos || !mix->cov) return SDMM_EINVAL;
    const int64_t chunk = default_chunk(opts);
    const int waves = default_waves(opts);
    if (chunk < 64 || chunk % 64 != 0 || !(waves == 1 || waves == 2 || waves == 4)) return SDMM_EINVAL;
    if ((int64_t)mix->n_cells + (n_samples + chunk - 1) / chunk > INT32_MAX) return SDMM_EINVAL;
    // per-chunk lane offsets are 32-bit byte offsets
    if (chunk_size_for(n_samples, chunk) * 4 > (int64_t)UINT32_MAX / 2) return SDMM_EINVAL;
    if (workspace_bytes < layout_for(mix->n_cells, opts->K, n_samples, chunk).total) return SDMM_ENOWORKSPACE;
    return SDMM_OK;
}

// graph cache: argument values -> instantiated graph
struct GraphKey {
    std::vector<char> bytes;
    bool operator<(const GraphKey& o) const { return bytes < o.bytes; }
};
static std::mutex g_graph_mu;
static std::map<GraphKey, hipGraphExec_t> g_graphs;

}  // namespace sdmm

using namespace sdmm;

extern "C" size_t sdmm_fit_workspace_size(int32_t n_cells, int32_t K, int64_t n_samples,
                                          const sdmm_fit_opts* opts)
{
    if (n_cells <= 0 || K < 1 || K > kMaxK || n_samples < 0 || !opts) return 0;
    return layout_for(n_cells, K, n_samples, default_chunk(opts)).total;
}

extern "C" int sdmm_fit_mixtures(const int64_t* cell_offsets, const float* samples, int64_t n_samples,
                                 const sdmm_mixtures* mix, const sdmm_em_state* state,
                                 const sdmm_fit_opts* opts, int32_t* cell_status, void* workspace,
                                 size_t workspace_bytes, void* stream)
{
    int rc = validate_fit_args(cell_offsets, samples, n_samples, mix, opts, cell_status, workspace, workspace_bytes);
    if (rc) return rc;
    if (!state || !state->s0 || !state->s2 || !state->sw || !state->step) return SDMM_EINVAL;
    if (opts->schedule != SDMM_SCHED_BATCHED && opts->schedule != SDMM_SCHED_PER_CELL) return SDMM_EINVAL;

    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    FitArgs a{cell_offsets, samples, n_samples, *mix, *state, *opts, cell_status,
              reinterpret_cast<char*>(workspace)};

    if (opts->schedule == SDMM_SCHED_PER_CELL) {
        std::vector<int64_t> host_off(mix->n_cells + 1);
        rc = check(hipMemcpyAsync(host_off.data(), cell_offsets, host_off.size() * sizeof(int64_t),
                                  hipMemcpyDeviceToHost, s));
        if (rc) return rc;
        rc = check(hipStreamSynchronize(s));
        if (rc) return rc;
        for (int c = 0; c < mix->n_cells; ++c)
            if (host_off[c + 1] < host_off[c] || host_off[c] < 0 || host_off[c + 1] > n_samples) return SDMM_EINVAL;
        return enqueue_fit(a, s, &host_off);
    }

    if (opts->use_graph && s != nullptr) {
        GraphKey key;
        key.bytes.resize(sizeof(FitArgs) + sizeof(void*));
        memcpy(key.bytes.data(), &a, sizeof(FitArgs));
        memcpy(key.bytes.data() + sizeof(FitArgs), &s, sizeof(void*));
        std::lock_guard<std::mutex> lk(g_graph_mu);
        auto it = g_graphs.find(key);
        if (it == g_graphs.end()) {
            hipGraph_t graph;
            rc = check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            if (rc) return rc;
            rc = enqueue_fit(a, s, nullptr);
            const hipError_t e2 = hipStreamEndCapture(s, &graph);
            if (rc) return rc;
            if ((rc = check(e2))) return rc;
            hipGraphExec_t exec;
            rc = check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            (void)hipGraphDestroy(graph);
            if (rc) return rc;
            it = g_graphs.emplace(key, exec).first;
        }
        return check(hipGraphLaunch(it->second, s));
    }
    return enqueue_fit(a, s, nullptr);
}

extern "C" const char* sdmm_status_string(int code)
{
    switch (code) {
        case SDMM_OK: return "ok";
        case SDMM_EINVAL: return "invalid argument";
        case SDMM_EDEVICE: return "HIP runtime error";
        case SDMM_ENOWORKSPACE: return "workspace too small";
    }
    return "unknown status";
}

extern "C" const char* sdmm_version(void) { return "sdmm-mi355x 0.1"; }
