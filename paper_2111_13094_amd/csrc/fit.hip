// fit.hip -- batched weighted MAP EM for spatio-directional Gaussian mixtures on gfx950.
//
// Method (Dodik et al., arXiv 2111.13094): statistics of Sec. 3.2 with tangent-space
// coordinates (Sec. 3.1), exp-map mean update and first-order covariance transfer
// (Sec. 3.2, 3.4), Robbins-Monro averaging and MAP updates (Sec. 4.3), one independent
// mixture per spatial cell updated only with at least min_samples vertices (Sec. 4.2).
//
// Kernels per call: setup (FP32 mirrors, status reset, offset checks; skipped when the
// previous call carried the mirrors), then per iteration: estep (one wave per work item)
// -> mstep (grouped cells).
//
// E-step work split: each cell's samples are cut, from the cell's first sample, into
// items of at most P = 2^ps samples; item j of cell c gets the record slot
// c + off[c]/P + j. For non-decreasing offsets these slots increase strictly from cell to
// cell and stay below C + ceil(N/P), so a wave recovers its cell from its slot by a
// 64-ary search over c + off[c]/P. The wave streams its item with one (sample,
// component) pair per lane (64/G sample slots x G component lanes) and writes one
// record (FP32, or FP64 for the FP64-sum pass); the M-step sums a cell's records in item
// order. A cell's results depend only on its own samples and P, and items of at most P
// samples keep the waves balanced.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "estep.hpp"
#include "mstep_math.hpp"
#include "timing.hpp"

namespace sdmm {

// ---------------------------------------------------------------------------------
// group helpers: a group of GM consecutive lanes (GM a power of two) handles one cell
// ---------------------------------------------------------------------------------
__device__ __forceinline__ double group_sum_d(double v, int GM)
{
    for (int o = 1; o < GM; o <<= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double group_max_d(double v, int GM)
{
    for (int o = 1; o < GM; o <<= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int group_or(int v, int GM)
{
    for (int o = 1; o < GM; o <<= 1) v |= __shfl_xor(v, o);
    return v;
}

// ---------------------------------------------------------------------------------
// One work group's check of the offsets, writing the control words: control[0] offsets
// non-decreasing within [0, N]; control[1] the most items in a cell; control[2] the
// record-tree levels launched. Run by the setup kernel's last block, or by the E-step
// launch's last block when the setup kernel does not run (carried mirrors).
// ---------------------------------------------------------------------------------
__device__ __forceinline__ void offsets_check_block(const int64_t* __restrict__ off, int64_t N, int C, int ps,
                                                    int32_t* __restrict__ control, int tree_max)
{
    __shared__ int bad, most;
    if (threadIdx.x == 0) bad = 0, most = 1;
    __syncthreads();
    // thread t checks cells t, t + blockDim, ...: consecutive threads read consecutive
    // offsets, eight cells' loads in flight per thread
    int b = 0;
    int64_t m = 1;
    for (int c0 = (int)threadIdx.x; c0 < C; c0 += 8 * (int)blockDim.x) {
        int64_t lo[8], hi[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int c = c0 + u * (int)blockDim.x;
            lo[u] = c < C ? off[c] : 0;
            hi[u] = c < C ? off[c + 1] : 0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            b |= hi[u] < lo[u];
            m = max(m, (hi[u] - lo[u] + (int64_t(1) << ps) - 1) >> ps);
        }
    }
    if (threadIdx.x == 0) b |= off[0] < 0 || off[C] > N;
    if (b) atomicOr(&bad, 1);
    atomicMax(&most, (int)min(m, (int64_t)INT32_MAX));
    __syncthreads();
    if (threadIdx.x == 0) {
        control[0] = bad ? 0 : 1;
        control[1] = most;
        control[2] = tree_max;
    }
}

// ---------------------------------------------------------------------------------
// setup: FP32 mirrors with the per-cell shift, status reset, per-cell flags; the last
// block checks that the offsets are non-decreasing within [0, N]
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void setup_kernel(const int64_t* __restrict__ off, int64_t N, int C, int K,
                                                    int GM, int ps, MixPtrs mix, float* __restrict__ mirror,
                                                    int32_t* __restrict__ flags, int32_t* __restrict__ status,
                                                    int32_t* __restrict__ arrive, int32_t* __restrict__ control,
                                                    int n_cell_blocks, int tree_max, int full)
{
    if ((int)blockIdx.x == n_cell_blocks) {
        offsets_check_block(off, N, C, ps, control, tree_max);
        return;
    }
    // one cell per group of GM lanes (64 / GM cells per wave), lane k % GM = component k:
    // the FP64 mirror construction then issues once for up to 64 components
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = (int)(t / GM);
    const int k = (int)(t % GM);
    const bool active = c < C && k < K;
    const int64_t g = (int64_t)c * K + k;
    double c2 = -INFINITY;
    bool ok = true;
    float m[kMirror];
    if (active) {
        ok = full ? write_mirror<true>(mix.pi[g], mix.mud + 3 * g, mix.mux + 3 * g, mix.cov + 15 * g, m, c2)
                  : write_mirror<false>(mix.pi[g], mix.mud + 3 * g, mix.mux + 3 * g, mix.cov + 15 * g, m, c2);
    }
    const double cmax = group_max_d(active && ok ? c2 : -INFINITY, GM);
    const int bad = group_or(active && !ok ? 1 : 0, GM);
    // the shift is an FP32 value, so adding it back in FP64 is exact
    const float shift = isfinite(cmax) ? (float)(cmax + 1.0) : 0.0f;
    if (full) {
        if (active) {
            set_mirror_shift<true>(m, c2, (double)shift, ok);
            store_mirror<true>(mirror + g * kMirror, m);
        }
    } else {
        // lite mirrors leave through LDS: a lane's own stores would touch 64 lines per
        // instruction (one 16-byte piece per component); read back in component order,
        // each store instruction writes eight components' lite mirrors whole
        __shared__ float4 stage[256][kMirrorLite / 4 + 1];
        if (active) {
            set_mirror_shift<false>(m, c2, (double)shift, ok);
#pragma unroll
            for (int q = 0; q < kMirrorLite / 4; ++q)
                stage[threadIdx.x][q] = make_float4(m[4 * q], m[4 * q + 1], m[4 * q + 2], m[4 * q + 3]);
        }
        __syncthreads();
        const int cpb = (int)blockDim.x / GM;  // cells per block
        const int c_lo = (int)blockIdx.x * cpb, c_hi = min(C, c_lo + cpb);
        const int64_t g_lo = (int64_t)c_lo * K;
        const int n = (c_hi - c_lo) * K * (kMirrorLite / 4);
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            const int comp = j / (kMirrorLite / 4), part = j % (kMirrorLite / 4);
            const int src = (comp / K) * GM + comp % K;
            reinterpret_cast<float4*>(mirror + (g_lo + comp) * kMirror)[part] = stage[src][part];
        }
    }
    if (c < C && k == 0) {
        status[c] = 0;
        arrive[c] = 0;
        const int64_t c0 = off[c], c1 = off[c + 1];
        flags[c] = ((c0 >= 0 && c1 >= c0 && c1 <= N) ? 0 : kFlagBadRange) | (bad ? kBadParams : 0);
    }
}

// ---------------------------------------------------------------------------------
// Work item of wave w of an E-step launch over the record slots [slot_lo, slot_hi):
// slot t = slot_lo + w, its cell by the 64-ary search, its item index t - first. False
// for a slot between two cells' items.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ bool wave_item(int64_t w, const int64_t* __restrict__ off, int64_t N, int C, int ps,
                                          int64_t slot_lo, int64_t slot_hi, int& c, int64_t& t, int64_t& s0,
                                          int64_t& s1, int64_t& n_items)
{
    t = slot_lo + w;
    if (t >= slot_hi) return false;
    c = find_slot_cell(off, C, ps, t);
    int64_t first;
    if (!cell_items(off, N, c, ps, first, n_items)) return false;
    const int64_t j = t - first;
    if (j < 0 || j >= n_items) return false;
    s0 = off[c] + (j << ps);
    s1 = min(s0 + (int64_t(1) << ps), off[c + 1]);
    return true;
}

// ---------------------------------------------------------------------------------
// XCD-aware work map of an E-step launch: work groups go to the eight XCDs in turn (group
// b to XCD b % 8), so the launch cuts its n_slots record slots into eight contiguous
// chunks and the groups of XCD x serve chunk x in order. The items of a cell (consecutive
// slots) then run on one XCD and share its L2: the cell's mirrors come from HBM once per
// cell instead of once per item. Returns the wave's slot offset, or -1 past its chunk.
// ---------------------------------------------------------------------------------
constexpr int kXcds = 8;

__host__ __device__ inline int64_t xcd_chunk(int64_t n_slots)
{
    return (n_slots + kXcds - 1) / kXcds;
}

__device__ __forceinline__ int64_t xcd_slot(int64_t group, int wpb, int wave, int64_t n_slots)
{
    const int64_t per = xcd_chunk(n_slots);
    const int64_t i = (group / kXcds) * wpb + wave;  // position in the chunk
    const int64_t w = (group % kXcds) * per + i;
    return (i < per && w < n_slots) ? w : -1;
}

// ---------------------------------------------------------------------------------
// E-step: one wave per work item (see wave_item), slots by the XCD-aware map
// ---------------------------------------------------------------------------------
// waves per SIMD the E-step needs: the plain-sum EM pass fits five (96 registers), which
// hides more of each item's start-up latency (cell search, mirror and first loads)
template <int ACC, bool JAC, bool ADJ>
constexpr int estep_min_waves()
{
    return (ACC == kAccPlain && !JAC && !ADJ) ? 5 : 1;
}

template <int G, int ACC, bool JAC, bool ADJ>
__global__ __launch_bounds__(256, (estep_min_waves<ACC, JAC, ADJ>())) void estep_kernel(const float* __restrict__ smp, int64_t N,
                                                    const int64_t* __restrict__ off, int C, int ps, int64_t slot_lo,
                                                    int64_t slot_hi, const float* __restrict__ mirror, int K, int PS,
                                                    void* __restrict__ records, int32_t* __restrict__ control,
                                                    int check_tree_max)
{
    // check_tree_max >= 0: the launch's last work group checks the offsets instead
    if (check_tree_max >= 0 && blockIdx.x == gridDim.x - 1) {
        offsets_check_block(off, N, C, ps, control, check_tree_max);
        return;
    }
    const int64_t w = xcd_slot(blockIdx.x, blockDim.x >> 6, __builtin_amdgcn_readfirstlane(threadIdx.x >> 6),
                               slot_hi - slot_lo);
    int c;
    int64_t t, s0, s1, n_items;
    if (w < 0 || !wave_item(w, off, N, C, ps, slot_lo, slot_hi, c, t, s0, s1, n_items)) return;
    estep_segment<G, ACC, JAC, ADJ>(smp, N, s0, s1, mirror + (int64_t)c * K * kMirror, K,
                                    static_cast<RecordT<ACC, ADJ>*>(records) + t * PS);
}

// FP64 adjoint pass (verification mode), same work map as estep_kernel
template <int G>
__global__ __launch_bounds__(256) void estep_adj64_kernel(const float* __restrict__ smp, int64_t N,
                                                          const int64_t* __restrict__ off, int C, int ps,
                                                          int64_t slot_lo, int64_t slot_hi,
                                                          const float* __restrict__ mirror, int K, int PS,
                                                          void* __restrict__ records, int32_t* __restrict__ control,
                                                          int check_tree_max)
{
    if (check_tree_max >= 0 && blockIdx.x == gridDim.x - 1) {
        offsets_check_block(off, N, C, ps, control, check_tree_max);
        return;
    }
    const int64_t w = xcd_slot(blockIdx.x, blockDim.x >> 6, __builtin_amdgcn_readfirstlane(threadIdx.x >> 6),
                               slot_hi - slot_lo);
    int c;
    int64_t t, s0, s1, n_items;
    if (w < 0 || !wave_item(w, off, N, C, ps, slot_lo, slot_hi, c, t, s0, s1, n_items)) return;
    estep_segment_adj64<G>(smp, N, s0, s1, mirror + (int64_t)c * K * kMirror, K, static_cast<double*>(records) + t * PS);
}

// ---------------------------------------------------------------------------------
// Lite mirror of component g for the next iteration (the EM passes read no more), written in
// place; with have, the update has already written it (from its own factorisation and
// frame, the values the stored parameters give again) and c2 is its unshifted constant,
// else it is built from the parameters.
// written in place (keeps the M-step's registers free), with the cell's shift from the
// group of GM lanes. `upd`: this lane's component was updated; the others keep their
// mirrors.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ void refresh_cell_mirror(const MixPtrs& mix, int64_t g, bool upd, float* __restrict__ mirror,
                                                    int GM, double c2 = -INFINITY, bool have = false)
{
    bool okm = true;
    float* out = mirror + g * kMirror;
    if (upd && !have) okm = write_mirror<false>(mix.pi[g], mix.mud + 3 * g, mix.mux + 3 * g, mix.cov + 15 * g, out, c2);
    if (!upd) c2 = -INFINITY;
    const double cmax = group_max_d((upd && okm) ? c2 : -INFINITY, GM);
    if (upd) set_mirror_shift<false>(out, c2, (double)(isfinite(cmax) ? (float)(cmax + 1.0) : 0.0f), okm);
}

// ---------------------------------------------------------------------------------
// The small inputs of one component's M-step besides its statistics: the cell's flags,
// the global offsets check, the cell's step count and blended weight sum, the
// component's carried S0 and current means. Loaded in one batch, so that a kernel can
// issue the loads before it sums the records and find them in registers afterwards (the
// carried S2 is loaded by the update itself, early in its chain).
// ---------------------------------------------------------------------------------
struct MstepIn {
    int fl, gok, step, range_ok;
    double sw, s0, mud[3], mux[3];
};

__device__ __forceinline__ MstepIn load_mstep_in(const int64_t* __restrict__ off, int64_t N, int c, int64_t g,
                                                 bool cell_ok, bool act, const int32_t* __restrict__ flags,
                                                 const int32_t* __restrict__ global_ok, const MixPtrs& mix,
                                                 const StatePtrs& st)
{
    MstepIn in;
    in.gok = *global_ok;
    in.fl = cell_ok ? flags[c] : 0;
    in.range_ok = cell_ok ? (off[c] >= 0 && off[c + 1] >= off[c] && off[c + 1] <= N) : 1;
    in.step = cell_ok ? st.step[c] : 0;
    in.sw = cell_ok ? st.sw[c] : 0.0;
    in.s0 = act ? st.s0[g] : 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        in.mud[d] = act ? mix.mud[3 * g + d] : 0.0;
        in.mux[d] = act ? mix.mux[3 * g + d] : 0.0;
    }
    return in;
}

// ---------------------------------------------------------------------------------
// M-step of one component (lane): from its cell's summed statistics (S: the component's,
// X: the cell's W, M and count of negative weights) and its other inputs `in` (loaded
// by load_mstep_in for the same c, k) it gates the cell, blends (Robbins-Monro) and
// updates in FP64, and optionally writes the next iteration's mirrors. Each group of G
// consecutive lanes holds the components of one cell (lane k % G = component k); every
// lane of the wave takes part (group reductions). c must be a valid cell index even where
// cell_ok is false.
// ---------------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ int64_t mstep_component(int c, int k, int K)
{
    return (int64_t)c * K + (k < K ? k : 0);
}

// M-step mode bits: write the next pass's mirrors; this is the call's first M-step write
// of the cell's status (no setup kernel reset it), so it assigns instead of or-ing
constexpr int kMRefresh = 1, kMFirstStatus = 2;

template <int G>
__device__ __forceinline__ void mstep_update(int c, int k, bool cell_ok, const double (&S)[kStats],
                                             const double (&X)[3], const MstepIn& in,
                                             int32_t* __restrict__ flags, const MixPtrs& mix,
                                             const StatePtrs& st, const DevOpts& o, float* __restrict__ mirror,
                                             int refresh_mirror, int32_t* __restrict__ status)
{
    constexpr int GM = G;
    const int K = o.K;
    // accurate covariance update: this M-step moves the weights and means only; the
    // mirrors it writes (new weights and means, previous covariances) drive the second
    // E-step pass, whose statistics accurate_mstep_kernel turns into the covariances
    const bool accurate = (o.flags & SDMM_FLAG_ACCURATE_SIGMA) != 0;
    const bool act = cell_ok && k < K;
    const int64_t g = mstep_component<G>(c, k, K);

    const double W = X[0], Mc = X[1], negs = X[2];
    int fin = isfinite(W);
    for (int s = 0; s < kStats; ++s) fin &= isfinite(S[s]) ? 1 : 0;
    const int notfin = group_or(act && !fin ? 1 : 0, GM) | (!isfinite(W) ? 1 : 0);
    int gate = 0, fl = 0;
    if (cell_ok) {
        fl = in.fl;
        if (negs > 0.0 || notfin || !in.range_ok || !in.gok) gate = kBadInput;
        else if (fl & kBadParams) gate = kBadParams;
        else if (Mc < (double)o.min_samples) gate = kSkippedFew;
        else if (!(W > 0.0)) gate = kSkippedZeroW;
    }
    const bool run = cell_ok && !gate;

    const int j = run ? in.step : 0;
    const double eta = rm_eta(o, j);
    const double beta = o.prior_mode == 0 ? eta / fmax(Mc, 1.0) : o.prior_scale;
    const double hW = j == 0 ? W : (1.0 - eta) * (run ? in.sw : 0.0) + eta * W;

    double hS0 = 0.0, hS1[5], hS2[15];
    if (run && act) {
        hS0 = j == 0 ? S[0] : (1.0 - eta) * in.s0 + eta * S[0];
        for (int d = 0; d < 5; ++d) hS1[d] = (j == 0 ? 1.0 : eta) * S[1 + d];
        for (int q = 0; q < 15; ++q) hS2[q] = j == 0 ? S[6 + q] : (1.0 - eta) * st.s2[g * 15 + q] + eta * S[6 + q];
    }
    const double bar0 = (run && act) ? hS0 / hW : 0.0;
    const double sum0 = group_sum_d(bar0, GM);

    int dead = 0, cholfail = 0;
    // the next mirror, written by the update when it replaces the covariance
    double c2m = -INFINITY;
    bool have_m = false;
    if (run && act) {
        const double pi_new = (beta * o.prior_q + bar0) / ((double)K * beta * o.prior_q + sum0);
        // with the accurate update the second pass forms the covariance
        component_map_update(hS0, hS1, hS2, hW, beta, bar0, o, !accurate, in.mud, in.mux, mix.mud + 3 * g,
                             mix.mux + 3 * g, mix.cov + 15 * g, st.s0 + g, st.s2 + 15 * g, dead, cholfail,
                             (refresh_mirror & kMRefresh) ? mirror + g * kMirror : nullptr, pi_new, c2m, have_m);
        mix.pi[g] = pi_new;
    }
    const int any_dead = group_or(dead, GM), any_chol = group_or(cholfail, GM);
    // for the next iteration, or the next call with carried mirrors
    if (refresh_mirror & kMRefresh) refresh_cell_mirror(mix, g, run && act, mirror, GM, c2m, have_m);
    if (cell_ok && k == 0) {
        if (accurate) flags[c] = gate ? (fl & ~kFlagStepped) : (fl | kFlagStepped);
        const int prev = (refresh_mirror & kMFirstStatus) ? 0 : status[c];
        if (gate) {
            status[c] = prev | gate;
        } else {
            st.sw[c] = hW;
            st.step[c] = j + 1;
            status[c] = prev | (any_dead ? kDeadComponent : 0) | (any_chol ? kCholFailKeptPrev : 0);
        }
    }
}

// M-step of one cell by one wave: all 64 lanes sum the cell's records (in item order,
// column-parallel), then lanes k < G (lane k = component k) update. cell_ok must be
// uniform over the wave.
template <int G, typename RT>
__device__ __forceinline__ void mstep_cell(const int64_t* __restrict__ off, int64_t N, int c, bool cell_ok, int ps,
                                           bool tree, const RT* __restrict__ records, int PS,
                                           int32_t* __restrict__ flags, const int32_t* __restrict__ global_ok,
                                           const MixPtrs& mix, const StatePtrs& st, const DevOpts& o,
                                           float* __restrict__ mirror, int refresh_mirror,
                                           int32_t* __restrict__ status)
{
    const int lane = threadIdx.x & 63;
    const bool lane_ok = cell_ok && lane < G;
    const MstepIn in = load_mstep_in(off, N, c, mstep_component<G>(c, lane, o.K), lane_ok, lane_ok && lane < o.K,
                                     flags, global_ok, mix, st);
    double S[kStats], X[3];
    int64_t first = 0, n_items = 0;
    const bool have = cell_ok && cell_items(off, N, c, ps, first, n_items);
    // after the record tree (batched and per-cell schedules) only the top leaders remain
    const int lv = tree && *global_ok ? tree_levels_done(global_ok) : 0;
    sum_cell_records<G, kStats, 3>(records, first, have ? n_items : 0, PS, kTreeLog2R * lv, S, X);
    mstep_update<G>(c, lane, lane_ok, S, X, in, flags, mix, st, o, mirror, refresh_mirror, status);
}

// M-step of cells [cell_lo, cell_lo + n_cells), one cell per wave
template <int G, typename RT>
__global__ __launch_bounds__(256) void mstep_kernel(const int64_t* __restrict__ off, int64_t N, int ps,
                                                    const void* __restrict__ records, int PS,
                                                    int32_t* __restrict__ flags,
                                                    const int32_t* __restrict__ global_ok, MixPtrs mix,
                                                    StatePtrs st, DevOpts o, float* __restrict__ mirror,
                                                    int refresh_mirror, int32_t* __restrict__ status,
                                                    int cell_lo, int n_cells)
{
    const int cl = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool cell_ok = cl < n_cells;
    mstep_cell<G>(off, N, cell_lo + (cell_ok ? cl : 0), cell_ok, ps, true, static_cast<const RT*>(records), PS, flags, global_ok, mix, st, o,
                  mirror, refresh_mirror, status);
}

// M-step of cells [cell_lo, cell_lo + n_cells) after the record tree, 64 / G cells per
// work group of 64 / G waves. Wave w sums the records of the group's cell w over all 64
// lanes into LDS; then one wave updates every component of the group's cells, lane
// w * G + k = component k of cell w. The FP64 update, which needs one lane per
// component, then issues once for 64 components instead of once per cell. The sums and
// the update are those of mstep_kernel, so both give the same results.
template <int G, typename RT>
__global__ __launch_bounds__(64 * (64 / G), G <= 16 ? 4 : 1) void mstep_packed_kernel(
    const int64_t* __restrict__ off, int64_t N, int ps, const void* __restrict__ records, int PS,
    int32_t* __restrict__ flags, const int32_t* __restrict__ global_ok, MixPtrs mix, StatePtrs st, DevOpts o,
    float* __restrict__ mirror, int refresh_mirror, int32_t* __restrict__ status, int cell_lo, int n_cells)
{
    constexpr int NCW = 64 / G, NCOL = kStats * G + 3, NQ = (NCOL + 63) / 64;
    __shared__ double cols[NCW][NCOL];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int cb = blockIdx.x * NCW;
    // the updating wave's other inputs, loaded before the record sums so that their
    // latency overlaps them
    const int slot = lane / G, k = lane % G;
    const int cu = cb + slot;
    const bool uok = w == 0 && cu < n_cells;
    const int cuc = cell_lo + (cu < n_cells ? cu : 0);
    MstepIn in{};
    if (w == 0)
        in = load_mstep_in(off, N, cuc, mstep_component<G>(cuc, k, o.K), uok, uok && k < o.K, flags, global_ok, mix,
                           st);
    {
        const int cl = cb + w;
        const bool ok = cl < n_cells;
        const int c = cell_lo + (ok ? cl : 0);
        int64_t first = 0, n_items = 0;
        const bool have = ok && cell_items(off, N, c, ps, first, n_items);
        const int lv = *global_ok ? tree_levels_done(global_ok) : 0;
        double v[NQ];
        // six FP32 (three FP64) records per round trip, which leaves room for the
        // prefetched update inputs
        sum_cell_columns<G, kStats, 3, 3>(static_cast<const RT*>(records), first, have ? n_items : 0, PS,
                                          kTreeLog2R * lv, v);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (q * 64 + lane < NCOL) cols[w][q * 64 + lane] = v[q];
    }
    __syncthreads();
    if (w != 0) return;
    double S[kStats], X[3];
#pragma unroll
    for (int s = 0; s < kStats; ++s) S[s] = cols[slot][s * G + k];
#pragma unroll
    for (int i = 0; i < 3; ++i) X[i] = cols[slot][kStats * G + i];
    mstep_update<G>(cuc, k, uok, S, X, in, flags, mix, st, o, mirror, refresh_mirror, status);
}

// ---------------------------------------------------------------------------------
// Accurate covariance update (Sec. 3.2: the second moment in the new mean's tangent
// space, with responsibilities from the densities in that tangent space). Per iteration:
// E-step, record tree, M-step for the weights and means only (it writes mirrors of the new
// weights and means with the previous covariances and marks the cells it stepped), the
// same E-step pass again on those mirrors (S0', S2' about the new means), its record tree,
// then accurate_mstep_kernel, one wave per cell:
//   Sigma = (beta B + S2' / W) / (beta a + S0' / W), beta = 1 / M unless fixed (eta = 1),
// a Cholesky check (the previous covariance is kept if it fails), carried S0 = S0' and
// S2 = S2', and the mirrors for the next iteration. Components dead in the first M-step
// keep what it left; one whose S0' / W is at or below the dead threshold keeps its
// covariance and flags the cell as dead. Cells the first M-step did not step are skipped.
// ---------------------------------------------------------------------------------
template <int G, typename RT>
__global__ __launch_bounds__(256) void accurate_mstep_kernel(const int64_t* __restrict__ off, int64_t N, int ps,
                                                             const void* __restrict__ records, int PS,
                                                             const int32_t* __restrict__ flags,
                                                             const int32_t* __restrict__ global_ok, MixPtrs mix,
                                                             StatePtrs st, DevOpts o, float* __restrict__ mirror,
                                                             int refresh_mirror, int32_t* __restrict__ status,
                                                             int cell_lo, int n_cells)
{
    const int cl = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (cl >= n_cells) return;
    const int c = cell_lo + cl;
    const int K = o.K;
    const int k = threadIdx.x & 63;
    const bool stepped = (flags[c] & kFlagStepped) != 0;  // uniform over the wave
    int64_t first = 0, n_items = 0;
    const bool have = stepped && cell_items(off, N, c, ps, first, n_items);
    const int lv = *global_ok ? tree_levels_done(global_ok) : 0;
    double S[kStats], X[3];
    sum_cell_records<G, kStats, 3>(static_cast<const RT*>(records), first, have ? n_items : 0, PS, kTreeLog2R * lv, S,
                                   X);
    const bool act = have && k < K;
    const int64_t g = (int64_t)c * K + (k < K ? k : 0);
    int dead = 0, cholfail = 0;
    if (act && st.s0[g] / st.sw[c] > o.dead_threshold) {  // else dead in the first M-step
        const double W = X[0], bar0 = S[0] / W;
        st.s0[g] = S[0];
        for (int q = 0; q < 15; ++q) st.s2[g * 15 + q] = S[6 + q];
        if (!(bar0 > o.dead_threshold)) {
            dead = 1;
        } else {
            const double beta = o.prior_mode == 0 ? 1.0 / fmax(X[1], 1.0) : o.prior_scale;
            const double iden = 1.0 / (beta * o.prior_a + bar0), iW = 1.0 / W;
            double Sig[15], Lt[15];
            for (int d = 0; d < 5; ++d)
                for (int e = 0; e <= d; ++e) {
                    double v = S[6 + tri(d, e)] * iW;
                    if (d == e) v += beta * o.prior_b[d];
                    Sig[tri(d, e)] = v * iden;
                }
            if (chol64<5>(Sig, Lt)) {
                for (int q = 0; q < 15; ++q) mix.cov[g * 15 + q] = Sig[q];
            } else {
                cholfail = 1;
            }
        }
    }
    const int any_dead = group_or(dead, G), any_chol = group_or(cholfail, G);
    if (refresh_mirror & kMRefresh) refresh_cell_mirror(mix, g, act, mirror, G);
    if (have && k == 0) status[c] |= (any_dead ? kDeadComponent : 0) | (any_chol ? kCholFailKeptPrev : 0);
}

// ---------------------------------------------------------------------------------
// Fused E+M: one wave per record slot as in estep_kernel; after writing its record a
// wave counts itself into the cell's arrival counter (device-scope release before,
// acquire after), and the wave that completes the count runs the cell's M-step on its
// wave and resets the counter for the next launch. Every cell has at least
// one item, so every cell gets its M-step. Offsets that are not non-decreasing within
// [0, N] (checked by the setup kernel) turn every cell into BAD_INPUT.
// ---------------------------------------------------------------------------------
template <int G, int ACC, bool JAC>
__global__ __launch_bounds__(256) void fused_kernel(const float* __restrict__ smp, int64_t N,
                                                    const int64_t* __restrict__ off, int C, int ps,
                                                    int64_t slot_hi, const float* __restrict__ mirror_in, int K,
                                                    int PS, void* __restrict__ records_v,
                                                    int32_t* __restrict__ arrive, int32_t* __restrict__ flags,
                                                    const int32_t* __restrict__ global_ok, MixPtrs mix, StatePtrs st,
                                                    DevOpts o, float* __restrict__ mirror, int refresh_mirror,
                                                    int32_t* __restrict__ status)
{
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (!*global_ok) {
        if (w < C && lane == 0) status[w] = kBadInput;
        return;
    }
    int c;
    int64_t t, s0, s1, n_items;
    if (!wave_item(w, off, N, C, ps, 0, slot_hi, c, t, s0, s1, n_items)) return;
    RecordT<ACC, false>* records = static_cast<RecordT<ACC, false>*>(records_v);
    estep_segment<G, ACC, JAC, false>(smp, N, s0, s1, mirror_in + (int64_t)c * K * kMirror, K, records + t * PS);
    __threadfence();
    int done = 0;
    if (lane == 0) done = atomicAdd(arrive + c, 1) == (int)n_items - 1;
    if (!__builtin_amdgcn_readfirstlane(done)) return;
    __threadfence();
    // no record tree here: the completing wave sums all of the cell's records itself
    mstep_cell<G>(off, N, c, true, ps, false, records, PS, flags, global_ok, mix, st, o, mirror, refresh_mirror,
                  status);
    if (lane == 0) arrive[c] = 0;
}

// ---------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------
template <int G, bool ADJ>
static EstepFn estep_for_g(int acc, bool jac)
{
    if constexpr (ADJ) {
        if (acc == kAccPlain) return estep_kernel<G, kAccPlain, false, true>;
        return estep_kernel<G, kAccTwoSum, false, true>;
    } else {
        if (jac) {
            if (acc == kAccPlain) return estep_kernel<G, kAccPlain, true, false>;
            if (acc == kAccFp64) return estep_kernel<G, kAccFp64, true, false>;
            return estep_kernel<G, kAccTwoSum, true, false>;
        }
        if (acc == kAccPlain) return estep_kernel<G, kAccPlain, false, false>;
        if (acc == kAccFp64) return estep_kernel<G, kAccFp64, false, false>;
        return estep_kernel<G, kAccTwoSum, false, false>;
    }
}

typedef void (*FusedFn)(const float*, int64_t, const int64_t*, int, int, int64_t, const float*, int, int,
                        void*, int32_t*, int32_t*, const int32_t*, MixPtrs, StatePtrs, DevOpts, float*, int,
                        int32_t*);
typedef void (*MstepFn)(const int64_t*, int64_t, int, const void*, int, int32_t*, const int32_t*, MixPtrs,
                        StatePtrs, DevOpts, float*, int, int32_t*, int, int);
typedef void (*AccMstepFn)(const int64_t*, int64_t, int, const void*, int, const int32_t*, const int32_t*, MixPtrs,
                           StatePtrs, DevOpts, float*, int, int32_t*, int, int);

template <typename RT>
static AccMstepFn accurate_mstep_function_t(int G)
{
    switch (G) {
        case 4: return accurate_mstep_kernel<4, RT>;
        case 8: return accurate_mstep_kernel<8, RT>;
        case 16: return accurate_mstep_kernel<16, RT>;
        case 32: return accurate_mstep_kernel<32, RT>;
        case 64: return accurate_mstep_kernel<64, RT>;
    }
    return nullptr;
}

// rec32: FP32 records (see RecordT)
static AccMstepFn accurate_mstep_function(int G, bool rec32)
{
    return rec32 ? accurate_mstep_function_t<float>(G) : accurate_mstep_function_t<double>(G);
}

template <typename RT>
static MstepFn mstep_packed_function_t(int G)
{
    switch (G) {
        case 4: return mstep_packed_kernel<4, RT>;
        case 8: return mstep_packed_kernel<8, RT>;
        case 16: return mstep_packed_kernel<16, RT>;
        case 32: return mstep_packed_kernel<32, RT>;
        case 64: return mstep_packed_kernel<64, RT>;
    }
    return nullptr;
}

// rec32: FP32 records (see RecordT)
static MstepFn mstep_packed_function(int G, bool rec32)
{
    return rec32 ? mstep_packed_function_t<float>(G) : mstep_packed_function_t<double>(G);
}

template <typename RT>
static MstepFn mstep_function_t(int G)
{
    switch (G) {
        case 4: return mstep_kernel<4, RT>;
        case 8: return mstep_kernel<8, RT>;
        case 16: return mstep_kernel<16, RT>;
        case 32: return mstep_kernel<32, RT>;
        case 64: return mstep_kernel<64, RT>;
    }
    return nullptr;
}

// rec32: FP32 records (see RecordT)
static MstepFn mstep_function(int G, bool rec32)
{
    return rec32 ? mstep_function_t<float>(G) : mstep_function_t<double>(G);
}

template <int G>
static FusedFn fused_for_g(int acc, bool jac)
{
    if (jac) {
        if (acc == kAccPlain) return fused_kernel<G, kAccPlain, true>;
        if (acc == kAccFp64) return fused_kernel<G, kAccFp64, true>;
        return fused_kernel<G, kAccTwoSum, true>;
    }
    if (acc == kAccPlain) return fused_kernel<G, kAccPlain, false>;
    if (acc == kAccFp64) return fused_kernel<G, kAccFp64, false>;
    return fused_kernel<G, kAccTwoSum, false>;
}

static FusedFn fused_function(int G, int acc, bool jac)
{
    switch (G) {
        case 4: return fused_for_g<4>(acc, jac);
        case 8: return fused_for_g<8>(acc, jac);
        case 16: return fused_for_g<16>(acc, jac);
        case 32: return fused_for_g<32>(acc, jac);
        case 64: return fused_for_g<64>(acc, jac);
    }
    return nullptr;
}

EstepFn adj64_function(int G)
{
    switch (G) {
        case 4: return estep_adj64_kernel<4>;
        case 8: return estep_adj64_kernel<8>;
        case 16: return estep_adj64_kernel<16>;
        case 32: return estep_adj64_kernel<32>;
        case 64: return estep_adj64_kernel<64>;
    }
    return nullptr;
}

EstepFn estep_function(int G, int acc, bool jac, bool adj)
{
    switch (G) {
        case 4: return adj ? estep_for_g<4, true>(acc, jac) : estep_for_g<4, false>(acc, jac);
        case 8: return adj ? estep_for_g<8, true>(acc, jac) : estep_for_g<8, false>(acc, jac);
        case 16: return adj ? estep_for_g<16, true>(acc, jac) : estep_for_g<16, false>(acc, jac);
        case 32: return adj ? estep_for_g<32, true>(acc, jac) : estep_for_g<32, false>(acc, jac);
        case 64: return adj ? estep_for_g<64, true>(acc, jac) : estep_for_g<64, false>(acc, jac);
    }
    return nullptr;
}

void launch_setup(const int64_t* off, int64_t N, const sdmm_mixtures& mix, int32_t* status, char* ws, const Layout& L,
                  hipStream_t s, bool full)
{
    const int C = mix.n_cells, K = mix.K;
    const int GM = group_pow2(K);
    const int blocks = (int)(((int64_t)C * GM + 255) / 256);  // one cell per GM lanes
    const MixPtrs mp{mix.weights, mix.mean_dir, mix.mean_pos, mix.cov};
    setup_kernel<<<blocks + 1, 256, 0, s>>>(off, N, C, K, GM, L.ps, mp, reinterpret_cast<float*>(ws + L.mirror),
                                            reinterpret_cast<int32_t*>(ws + L.flags), status,
                                            reinterpret_cast<int32_t*>(ws + L.arrive),
                                            reinterpret_cast<int32_t*>(ws + L.global_ok), blocks,
                                            tree_levels_launched(N, L.P, L.max_cell), full ? 1 : 0);
}

void launch_estep(EstepFn est, const float* smp, int64_t N, const int64_t* off, int C, int K, const Layout& L,
                  int64_t slot_lo, int64_t slot_hi, int PS, char* ws, hipStream_t s, bool check)
{
    const int64_t waves = slot_hi - slot_lo;
    if (waves <= 0 && !check) return;
    // the XCD-aware map (xcd_slot): eight chunks of xcd_chunk(waves) slots, each served by
    // its XCD's groups; with the offsets check, one more work group (past every work item)
    // runs it
    const int64_t per = xcd_chunk(std::max<int64_t>(waves, 0));
    const unsigned blocks = (unsigned)(kXcds * ((per + L.wpb - 1) / L.wpb)) + (check ? 1u : 0u);
    hipLaunchKernelGGL(est, dim3(blocks), dim3(64 * L.wpb), 0, s, smp, N, off, C, L.ps, slot_lo, slot_hi,
                       reinterpret_cast<const float*>(ws + L.mirror), K, PS, static_cast<void*>(ws + L.records),
                       reinterpret_cast<int32_t*>(ws + L.global_ok),
                       check ? tree_levels_launched(N, L.P, L.max_cell) : -1);
}

typedef void (*TreeFn)(const int64_t*, int64_t, int, int, int, int64_t, int64_t, const int32_t*, void*, int);

template <int NS, int NX, typename RT>
static TreeFn tree_function(int G)
{
    switch (G) {
        case 4: return tree_kernel<4, NS, NX, RT>;
        case 8: return tree_kernel<8, NS, NX, RT>;
        case 16: return tree_kernel<16, NS, NX, RT>;
        case 32: return tree_kernel<32, NS, NX, RT>;
        case 64: return tree_kernel<64, NS, NX, RT>;
    }
    return nullptr;
}

void launch_tree(TreePass pass, const int64_t* off, int64_t N, int C, int K, const Layout& L, int cell, int64_t c0,
                 int64_t c1, char* ws, hipStream_t s, bool rec32)
{
    const int G = group_for(K);
    const TreeFn fn = pass == kTreeGrad ? tree_function<kStats + 2, 4, double>(G)
                      : rec32           ? tree_function<kStats, 3, float>(G)
                                        : tree_function<kStats, 3, double>(G);
    const int PS = pass == kTreeGrad ? L.ps_grad : L.ps_fit;
    // a bound from the caller's largest cell (else all samples in one cell); the device
    // skips levels no cell needs
    const int levels = tree_levels_launched(N, L.P, L.max_cell);
    for (int level = 1; level <= levels; ++level) {
        const int psl = L.ps + kTreeLog2R * level;
        int64_t lo = 0, hi = (int64_t)C + ((N + (int64_t(1) << psl) - 1) >> psl);
        if (cell >= 0) {  // one cell's leaders only
            lo = cell + (c0 >> psl);
            hi = lo + (c1 > c0 ? (c1 - c0 + (int64_t(1) << psl) - 1) >> psl : 1);
        }
        const int64_t blocks = std::min<int64_t>((hi - lo + 3) / 4, 256);  // grid-stride: at most 1024 waves
        hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(256), 0, s, off, N, C, L.ps, level, lo, hi,
                           reinterpret_cast<const int32_t*>(ws + L.global_ok), static_cast<void*>(ws + L.records), PS);
    }
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

// carry_in: the workspace already holds mirrors of the current parameters and the cells'
// parameter flags (written by the previous call's last M-step), so no setup kernel runs:
// the first E-step launch checks the offsets and the first M-step assigns the statuses.
// carry_out: the last M-step writes the mirrors for the next call. Batched schedule only.
static int enqueue_fit(const FitArgs& a, hipStream_t s, const std::vector<int64_t>* host_off, bool carry_in,
                       bool carry_out)
{
    const int C = a.mix.n_cells, K = a.opts.K;
    const int G = group_for(K);
    const Layout L = layout_for(C, K, a.N, &a.opts);
    const MixPtrs mp{a.mix.weights, a.mix.mean_dir, a.mix.mean_pos, a.mix.cov};
    const StatePtrs sp{a.st.s0, a.st.s2, a.st.sw, a.st.step};
    const DevOpts dopt = dev_opts(&a.opts);
    const int acc = (a.opts.flags & SDMM_FLAG_PLAIN_FP32) ? kAccPlain
                    : (a.opts.flags & SDMM_FLAG_FP64_SUMS) ? kAccFp64 : kAccTwoSum;
    const bool jac = (a.opts.flags & SDMM_FLAG_ESTEP_JACOBIAN) != 0;
    const bool accurate = (a.opts.flags & SDMM_FLAG_ACCURATE_SIGMA) != 0;
    // a lane's share of a work item fits one block of the compensated sums when the item
    // has at most kFoldEvery steps of 64 / G samples: no fold ever runs, the running total
    // stays zero, and the compensated pass is bit for bit the plain one, which needs fewer
    // registers
    const bool one_block = (L.P / (64 / G)) <= kFoldEvery;
    EstepFn est = estep_function(G, (acc == kAccTwoSum && one_block) ? kAccPlain : acc, jac, false);
    FusedFn fused = fused_function(G, acc, jac);
    const bool rec32 = acc != kAccFp64;  // record element type of these passes (RecordT)
    MstepFn mstep = mstep_function(G, rec32), mstep_packed = mstep_packed_function(G, rec32);
    AccMstepFn acc_mstep = accurate ? accurate_mstep_function(G, rec32) : nullptr;
    float* mirror = reinterpret_cast<float*>(a.ws + L.mirror);
    int32_t* flags = reinterpret_cast<int32_t*>(a.ws + L.flags);
    const int32_t* gok = reinterpret_cast<const int32_t*>(a.ws + L.global_ok);
    void* rec = static_cast<void*>(a.ws + L.records);

    // second E-step pass of the accurate update over record slots [lo, hi) on the mirrors
    // the first M-step wrote, then its record tree
    auto second_pass = [&](int64_t lo, int64_t hi, int cell, int64_t c0, int64_t c1) {
        {
            ScopedTimer tm(SDMM_TIMER_ACCURATE, s);
            launch_estep(est, a.smp, a.N, a.off, C, K, L, lo, hi, L.ps_fit, a.ws, s);
        }
        launch_tree(kTreeFit, a.off, a.N, C, K, L, cell, c0, c1, a.ws, s, rec32);
    };

    if (!carry_in) launch_setup(a.off, a.N, a.mix, a.status, a.ws, L, s, false);
    if (a.opts.schedule == SDMM_SCHED_STEPWISE) {
        launch_stepwise(a.off, a.smp, a.N, a.mix, a.st, a.opts, a.status, L, a.ws, s);
        return check(hipGetLastError());
    }
    for (int it = 0; it < a.opts.iters; ++it) {
        const int refresh = (it + 1 < a.opts.iters || carry_out) ? kMRefresh : 0;
        const int first_status = (carry_in && it == 0) ? kMFirstStatus : 0;
        // with the accurate update the first M-step always writes mirrors (for the second
        // pass) and the accurate M-step those of the next iteration
        const int refresh1 = (accurate ? kMRefresh : refresh) | first_status;
        if (a.opts.schedule == SDMM_SCHED_PER_CELL) {
            // host_off is empty when the offsets failed the host check: the M-steps then
            // only report BAD_INPUT (the setup kernel's check agrees)
            for (int c = 0; c < C; ++c) {
                int64_t c0 = 0, c1 = 0, first = 0, n_items = 0;
                if (!host_off->empty()) {
                    c0 = (*host_off)[c];
                    c1 = (*host_off)[c + 1];
                    first = c + (c0 >> L.ps);
                    n_items = c1 > c0 ? (c1 - c0 + L.P - 1) >> L.ps : 1;
                    launch_estep(est, a.smp, a.N, a.off, C, K, L, first, first + n_items, L.ps_fit, a.ws, s);
                    launch_tree(kTreeFit, a.off, a.N, C, K, L, c, c0, c1, a.ws, s, rec32);
                }
                hipLaunchKernelGGL(mstep, dim3(1), dim3(64), 0, s, a.off, a.N, L.ps, rec, L.ps_fit, flags, gok, mp, sp,
                                   dopt, mirror, refresh1, a.status, c, 1);
                if (accurate) {
                    if (!host_off->empty()) second_pass(first, first + n_items, c, c0, c1);
                    hipLaunchKernelGGL(acc_mstep, dim3(1), dim3(64), 0, s, a.off, a.N, L.ps, rec, L.ps_fit, flags, gok,
                                       mp, sp, dopt, mirror, refresh, a.status, c, 1);
                }
            }
        } else if (a.opts.schedule == SDMM_SCHED_BATCHED) {
            {
                ScopedTimer tm(SDMM_TIMER_ESTEP, s);
                launch_estep(est, a.smp, a.N, a.off, C, K, L, 0, (int64_t)C + L.W, L.ps_fit, a.ws, s,
                             carry_in && it == 0);
            }
            launch_tree(kTreeFit, a.off, a.N, C, K, L, -1, 0, 0, a.ws, s, rec32);
            {
                ScopedTimer tm(SDMM_TIMER_MSTEP, s);
                const int ncw = 64 / G;  // cells per work group
                hipLaunchKernelGGL(mstep_packed, dim3((C + ncw - 1) / ncw), dim3(64 * ncw), 0, s, a.off, a.N, L.ps,
                                   rec, L.ps_fit, flags, gok, mp, sp, dopt, mirror, refresh1, a.status, 0, C);
            }
            if (accurate) {
                second_pass(0, (int64_t)C + L.W, -1, 0, 0);
                hipLaunchKernelGGL(acc_mstep, dim3((C + 3) / 4), dim3(256), 0, s, a.off, a.N, L.ps, rec, L.ps_fit,
                                   flags, gok, mp, sp, dopt, mirror, refresh, a.status, 0, C);
            }
        } else {
            ScopedTimer tm(SDMM_TIMER_ESTEP, s);
            const int64_t slots = (int64_t)C + L.W;
            hipLaunchKernelGGL(fused, dim3((unsigned)((slots + 3) / 4)), dim3(256), 0, s, a.smp, a.N, a.off, C, L.ps,
                               slots, mirror, K, L.ps_fit, rec, reinterpret_cast<int32_t*>(a.ws + L.arrive), flags,
                               gok, mp, sp, dopt, mirror, refresh, a.status);
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
    if (opts->min_range < 0 || opts->max_ranges < 0 || opts->max_ranges > (1 << 20)) return SDMM_EINVAL;
    if (opts->waves_per_block < 0 || opts->waves_per_block > 4 || opts->waves_per_block == 3 ||
        opts->max_cell_samples < 0)
        return SDMM_EINVAL;
    if (opts->flags & ~(SDMM_FLAG_ESTEP_JACOBIAN | SDMM_FLAG_PLAIN_FP32 | SDMM_FLAG_FP64_SUMS | SDMM_FLAG_ACCURATE_SIGMA |
                        SDMM_FLAG_CARRY_MIRRORS))
        return SDMM_EINVAL;

    const Layout L = layout_for(mix->n_cells, opts->K, n_samples, opts);
    // lane offsets inside a segment are 32-bit byte offsets; record slots are int32
    if (L.P * 4 > (int64_t)INT32_MAX || (int64_t)mix->n_cells + L.W > INT32_MAX) return SDMM_EINVAL;
    if (workspace_bytes < L.total) return SDMM_ENOWORKSPACE;
    return SDMM_OK;
}

// graph cache: argument values -> instantiated graph
struct GraphKey {
    std::vector<char> bytes;
    bool operator<(const GraphKey& o) const { return bytes < o.bytes; }
};
static std::mutex g_graph_mu;
static std::map<GraphKey, hipGraphExec_t> g_graphs;

// workspace -> the mixture arrays whose current parameters its mirrors hold
struct CarryTag {
    const void *w, *md, *mx, *cv;
    int32_t C, K;
};
static std::mutex g_carry_mu;
static std::map<const void*, CarryTag> g_carry;

bool mirrors_carried(const void* ws, const sdmm_mixtures& mix)
{
    std::lock_guard<std::mutex> lk(g_carry_mu);
    auto it = g_carry.find(ws);
    if (it == g_carry.end()) return false;
    const CarryTag& t = it->second;
    return t.w == mix.weights && t.md == mix.mean_dir && t.mx == mix.mean_pos && t.cv == mix.cov &&
           t.C == mix.n_cells && t.K == mix.K;
}

void mark_mirrors(const void* ws, const sdmm_mixtures& mix, bool carried)
{
    std::lock_guard<std::mutex> lk(g_carry_mu);
    if (carried)
        g_carry[ws] = CarryTag{mix.weights, mix.mean_dir, mix.mean_pos, mix.cov, mix.n_cells, mix.K};
    else
        g_carry.erase(ws);
}

}  // namespace sdmm

using namespace sdmm;

extern "C" size_t sdmm_fit_workspace_size(int32_t n_cells, int32_t K, int64_t n_samples,
                                          const sdmm_fit_opts* opts)
{
    if (n_cells <= 0 || K < 1 || K > kMaxK || n_samples < 0 || !opts) return 0;
    return layout_for(n_cells, K, n_samples, opts).total;
}

extern "C" int sdmm_fit_mixtures(const int64_t* cell_offsets, const float* samples, int64_t n_samples,
                                 const sdmm_mixtures* mix, const sdmm_em_state* state,
                                 const sdmm_fit_opts* opts, int32_t* cell_status, void* workspace,
                                 size_t workspace_bytes, void* stream)
{
    int rc = validate_fit_args(cell_offsets, samples, n_samples, mix, opts, cell_status, workspace, workspace_bytes);
    if (rc) return rc;
    if (!state || !state->s0 || !state->s2 || !state->sw || !state->step) return SDMM_EINVAL;
    if (opts->schedule != SDMM_SCHED_BATCHED && opts->schedule != SDMM_SCHED_PER_CELL &&
        opts->schedule != SDMM_SCHED_FUSED && opts->schedule != SDMM_SCHED_STEPWISE)
        return SDMM_EINVAL;
    // the accurate covariance update is defined for batch steps and has no fused or
    // stepwise form
    if ((opts->flags & SDMM_FLAG_ACCURATE_SIGMA) &&
        (opts->eta_mode != SDMM_ETA_CONSTANT || opts->eta != 1.0 || opts->schedule == SDMM_SCHED_FUSED ||
         opts->schedule == SDMM_SCHED_STEPWISE))
        return SDMM_EINVAL;

    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    FitArgs a{cell_offsets, samples, n_samples, *mix, *state, *opts, cell_status,
              reinterpret_cast<char*>(workspace)};
    // carried mirrors (batched schedule): reuse them when this workspace's last call wrote
    // them for these mixture arrays, and write them for the next call
    const bool carry_out = (opts->flags & SDMM_FLAG_CARRY_MIRRORS) && opts->schedule == SDMM_SCHED_BATCHED;
    const bool carry_in = carry_out && mirrors_carried(workspace, *mix);
    // the mark is taken down before any enqueue, so a failing call never leaves it up
    mark_mirrors(workspace, *mix, false);

    if (opts->schedule == SDMM_SCHED_PER_CELL) {
        std::vector<int64_t> host_off(mix->n_cells + 1);
        rc = check(hipMemcpyAsync(host_off.data(), cell_offsets, host_off.size() * sizeof(int64_t),
                                  hipMemcpyDeviceToHost, s));
        if (rc) return rc;
        rc = check(hipStreamSynchronize(s));
        if (rc) return rc;
        bool ok = host_off[0] >= 0 && host_off[mix->n_cells] <= n_samples;
        for (int c = 0; c < mix->n_cells && ok; ++c) ok = host_off[c + 1] >= host_off[c];
        if (!ok) host_off.clear();
        return enqueue_fit(a, s, &host_off, false, false);
    }

    if (opts->use_graph && s != nullptr) {
        GraphKey key;
        key.bytes.resize(sizeof(FitArgs) + sizeof(void*) + 1);
        memcpy(key.bytes.data(), &a, sizeof(FitArgs));
        memcpy(key.bytes.data() + sizeof(FitArgs), &s, sizeof(void*));
        key.bytes[sizeof(FitArgs) + sizeof(void*)] = carry_in ? 1 : 0;
        std::lock_guard<std::mutex> lk(g_graph_mu);
        auto it = g_graphs.find(key);
        if (it == g_graphs.end()) {
            hipGraph_t graph;
            rc = check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            if (rc) return rc;
            rc = enqueue_fit(a, s, nullptr, carry_in, carry_out);
            const hipError_t e2 = hipStreamEndCapture(s, &graph);
            if (rc) return rc;
            if ((rc = check(e2))) return rc;
            hipGraphExec_t exec;
            rc = check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            (void)hipGraphDestroy(graph);
            if (rc) return rc;
            it = g_graphs.emplace(key, exec).first;
        }
        rc = check(hipGraphLaunch(it->second, s));
        if (!rc && carry_out) mark_mirrors(workspace, *mix, true);
        return rc;
    }
    rc = enqueue_fit(a, s, nullptr, carry_in, carry_out);
    if (!rc && carry_out) mark_mirrors(workspace, *mix, true);
    return rc;
}

namespace sdmm {

// ---------------------------------------------------------------------------------
// The fit without a caller workspace, for callers that cannot allocate device memory
// (code under graph capture, serving loops). Its workspace is this file-scope array, one
// copy per device, held from the library's load to the end of the process. In host code
// the array's name only stands for the symbol: its device address comes from
// hipGetSymbolAddress, looked up once per device on the first call with that device
// current, and only that address is passed to kernels.
// ---------------------------------------------------------------------------------
static __device__ __align__(256) char scratch[SDMM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's scratch array (nullptr and an error code on
// failure)
static int scratch_for_current_device(char** out)
{
    *out = nullptr;
    int dev = 0;
    int rc = check(hipGetDevice(&dev));
    if (rc) return rc;
    if (dev < 0 || dev >= kMaxDevices) return SDMM_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        rc = check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (rc) return rc;
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return SDMM_OK;
}

}  // namespace sdmm

extern "C" int sdmm_fit_mixtures_noalloc(const int64_t* cell_offsets, const float* samples, int64_t n_samples,
                                         const sdmm_mixtures* mix, const sdmm_em_state* state,
                                         const sdmm_fit_opts* opts, int32_t* cell_status, void* stream)
{
    // the per-cell schedule copies the offsets to the host, and the graph cache
    // instantiates graphs: neither belongs in a call that must not allocate
    if (!opts || opts->schedule == SDMM_SCHED_PER_CELL || opts->use_graph) return SDMM_EINVAL;
    // the argument checks of sdmm_fit_mixtures, with the scratch array's size as the
    // workspace size (they only test the workspace pointer for null: cell_offsets
    // stands in for it here, before the device address is known)
    int rc = validate_fit_args(cell_offsets, samples, n_samples, mix, opts, cell_status, cell_offsets,
                               (size_t)SDMM_NOALLOC_SCRATCH_BYTES);
    if (rc) return rc;
    char* ws = nullptr;
    rc = scratch_for_current_device(&ws);
    if (rc) return rc;
    return sdmm_fit_mixtures(cell_offsets, samples, n_samples, mix, state, opts, cell_status, ws,
                             (size_t)SDMM_NOALLOC_SCRATCH_BYTES, stream);
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

extern "C" const char* sdmm_version(void) { return "sdmm-mi355x 0.2"; }
