// stepwise.hip -- stepwise (per-sample) EM on gfx950: the alternative to mini-batch EM that
// the paper weighs in Sec. 6 ("Mini-batch EM versus stepwise EM"; Cappe and Moulines 2009,
// weighted as in Vorba et al. 2014).
//
// One wave per cell, lane k = component k (the first G = K rounded up to a power of two
// lanes), FP64 throughout, samples in index order. Per sample with positive weight: the
// responsibilities under the current parameters (log map, quadratic form through the
// Cholesky factor, a log-sum-exp over the component lanes), the Robbins-Monro blend for
// the cell's sample counter, and the MAP update of component_map_update with a
// mini-batch of one (beta = eta unless fixed); then the component's frame, factor and log
// constant are rebuilt for the next sample. A fresh cell (step 0) first accumulates the
// statistics of its whole batch in the same sample order and takes one batch step. The chain is sequential within a cell; cells run in parallel, so
// the pass lasts as long as its largest cell: the per-sample reductions run within the
// component lanes (DPP) and every flag is a ballot.
#include "common.hpp"
#include "mstep_math.hpp"
#include "timing.hpp"

namespace sdmm {

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o);
    return v;
}

// an FP64 value of the lane given by a DPP pattern of the row (both halves moved)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, true),
                            __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, true));
}

// sum / maximum over each group of G consecutive lanes (every lane of a group gets it):
// DPP inside rows of 16 lanes, shuffles across rows
template <int G>
__device__ __forceinline__ double group_sum_fp64(double v)
{
    if constexpr (G >= 2) v += dpp_d<kDppXor1>(v);
    if constexpr (G >= 4) v += dpp_d<kDppXor2>(v);
    if constexpr (G >= 8) v += dpp_d<kDppHalfMirror>(v);
    if constexpr (G >= 16) v += dpp_d<kDppMirror>(v);
    if constexpr (G >= 32) v += __shfl_xor(v, 16);
    if constexpr (G >= 64) v += __shfl_xor(v, 32);
    return v;
}
template <int G>
__device__ __forceinline__ double group_max_fp64(double v)
{
    if constexpr (G >= 2) v = fmax(v, dpp_d<kDppXor1>(v));
    if constexpr (G >= 4) v = fmax(v, dpp_d<kDppXor2>(v));
    if constexpr (G >= 8) v = fmax(v, dpp_d<kDppHalfMirror>(v));
    if constexpr (G >= 16) v = fmax(v, dpp_d<kDppMirror>(v));
    if constexpr (G >= 32) v = fmax(v, __shfl_xor(v, 16));
    if constexpr (G >= 64) v = fmax(v, __shfl_xor(v, 32));
    return v;
}

// any lane of the wave
__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0; }

// a component prepared for the E-step: frame, positional mean, Cholesky factor with its
// reciprocal diagonal, log pi - log det L - (5/2) log 2 pi
struct Comp64 {
    double R[9], mx[3], L[15], rd[5], logc;
    bool ok;
};

__device__ inline void make_inert(Comp64& c)
{
    c.ok = false;
    c.logc = -INFINITY;
    for (int i = 0; i < 9; ++i) c.R[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int i = 0; i < 15; ++i) c.L[i] = 0.0;
    for (int d = 0; d < 5; ++d) c.L[tri(d, d)] = c.rd[d] = 1.0;
}

// the log constant from the weight and the factor
__device__ __forceinline__ void set_log_constant(Comp64& c, double pi)
{
    double ld = 0.0;
    for (int d = 0; d < 5; ++d) ld += log(c.L[tri(d, d)]);
    c.logc = log(pi) - ld - 2.5 * kLn2Pi;
}

__device__ inline void load_comp(const MixPtrs& mix, int64_t g, Comp64& c)
{
    const double pi = mix.pi[g];
    double mu[3];
    bool ok = isfinite(pi) && pi >= 0.0;
    for (int d = 0; d < 3; ++d) {
        mu[d] = mix.mud[3 * g + d];
        c.mx[d] = mix.mux[3 * g + d];
        ok = ok && isfinite(mu[d]) && isfinite(c.mx[d]);
    }
    ok = ok && chol64<5>(mix.cov + 15 * g, c.L);
    c.ok = ok;
    if (!ok) {
        make_inert(c);
        return;
    }
    frame64(mu, c.R);
    for (int d = 0; d < 5; ++d) c.rd[d] = 1.0 / c.L[tri(d, d)];
    set_log_constant(c, pi);
}

// tangent coordinates of a sample and the component's log density there
__device__ inline double comp_log_density(const Comp64& c, const double w[3], const double p[3], bool jac,
                                          double y[5])
{
    const double x = c.R[0] * w[0] + c.R[1] * w[1] + c.R[2] * w[2];
    const double yy = c.R[3] * w[0] + c.R[4] * w[1] + c.R[5] * w[2];
    const double z = c.R[6] * w[0] + c.R[7] * w[1] + c.R[8] * w[2];
    const double s = hypot(x, yy);
    if (s > 0.0) {
        const double f = atan2(s, z) / s;
        y[0] = f * x;
        y[1] = f * yy;
    } else {
        y[0] = z >= 0.0 ? 0.0 : kPi;  // the antipode maps to (pi, 0)
        y[1] = 0.0;
    }
    for (int d = 0; d < 3; ++d) y[2 + d] = p[d] - c.mx[d];
    double zz[5], q = 0.0;
    for (int d = 0; d < 5; ++d) {
        double v = y[d];
        for (int e = 0; e < d; ++e) v -= c.L[tri(d, e)] * zz[e];
        zz[d] = v * c.rd[d];
        q += zz[d] * zz[d];
    }
    double l = c.logc - 0.5 * q;
    if (jac) {
        const double r = hypot(y[0], y[1]);
        if (r > 0.0) l -= log(sin(r) / r);
    }
    return l;
}

template <int G>
__global__ __launch_bounds__(256) void stepwise_kernel(const int64_t* __restrict__ off, int64_t N,
                                                       const float* __restrict__ smp, int C, MixPtrs mix,
                                                       StatePtrs st, DevOpts o, int iters,
                                                       const int32_t* __restrict__ flags,
                                                       const int32_t* __restrict__ control,
                                                       int32_t* __restrict__ status)
{
    const int c = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (c >= C) return;
    const int K = o.K;
    const int k = threadIdx.x & 63;
    const bool act = k < K;
    const int64_t g = (int64_t)c * K + (act ? k : 0);
    const bool jac = (o.flags & SDMM_FLAG_ESTEP_JACOBIAN) != 0;
    int st_bits = 0;
    const int64_t i0 = off[c], i1 = off[c + 1];
    const bool range_ok = control[0] && !(flags[c] & kFlagBadRange);
    int j = st.step[c];
    double sw = st.sw[c];
    Comp64 cp;
    load_comp(mix, g, cp);
    for (int it = 0; it < iters; ++it) {
        // the cell gate over the whole batch, all 64 lanes
        bool bad = !range_ok;
        double Wt = 0.0, Mt = 0.0;
        if (range_ok) {
            for (int64_t i = i0 + k; i < i1; i += 64) {
                const float wi = smp[6 * N + i];
                bool b = wi < 0.0f;
                for (int a = 0; a < 7; ++a) b = b || !isfinite(smp[a * N + i]);
                bad = bad || b;
                Wt += (double)wi;
                Mt += wi > 0.0f ? 1.0 : 0.0;
            }
        }
        const bool any_bad = wave_any(bad);
        Wt = wave_sum_d(Wt);
        Mt = wave_sum_d(Mt);
        const bool badp = wave_any(act && !cp.ok);
        int gate = 0;
        if (any_bad) gate = kBadInput;
        else if (badp) gate = kBadParams;
        else if (Mt < (double)o.min_samples) gate = kSkippedFew;
        else if (!(Wt > 0.0)) gate = kSkippedZeroW;
        if (gate) {
            st_bits |= gate;
            break;
        }
        const bool fresh = j == 0;
        double S[21];
        double Wb = 0.0, Mb = 0.0;
        for (int q = 0; q < 21; ++q) S[q] = 0.0;
        bool stop = false;
        for (int64_t i = i0; i < i1 && !stop; ++i) {
            const double wi = (double)smp[6 * N + i];
            if (fresh) {
                Wb += wi;
                Mb += wi > 0.0 ? 1.0 : 0.0;
            } else if (!(wi > 0.0)) {
                continue;
            }
            const double w[3] = {(double)smp[i], (double)smp[N + i], (double)smp[2 * N + i]};
            const double p[3] = {(double)smp[3 * N + i], (double)smp[4 * N + i], (double)smp[5 * N + i]};
            double y[5];
            double l = comp_log_density(cp, w, p, jac, y);
            if (!act) l = -INFINITY;
            // the log-sum-exp over the component lanes (the first G lanes hold the cell's
            // components; the other groups of G lanes hold only inactive lanes)
            const double lmax = group_max_fp64<G>(l);
            const double e = act ? exp(l - lmax) : 0.0;
            const double den = group_sum_fp64<G>(e);
            const double wr = act ? wi * (e / den) : 0.0;
            if (fresh) {
                S[0] += wr;
                for (int d = 0; d < 5; ++d) {
                    S[1 + d] += wr * y[d];
                    for (int f = 0; f <= d; ++f) S[6 + tri(d, f)] += wr * y[d] * y[f];
                }
                continue;
            }
            // a mini-batch of one
            S[0] = wr;
            for (int d = 0; d < 5; ++d) {
                S[1 + d] = wr * y[d];
                for (int f = 0; f <= d; ++f) S[6 + tri(d, f)] = wr * y[d] * y[f];
            }
            Wb = wi;
            Mb = 1.0;
            bool fin = isfinite(Wb);
            for (int q = 0; q < 21; ++q) fin = fin && isfinite(S[q]);
            if (wave_any(act && !fin)) {
                st_bits |= kBadInput;
                stop = true;
                break;
            }
            const double eta = rm_eta(o, j);
            const double beta = o.prior_mode == 0 ? eta / fmax(Mb, 1.0) : o.prior_scale;
            const double hW = (1.0 - eta) * sw + eta * Wb;
            double hS0 = 0.0, hS1[5], hS2[15];
            if (act) {
                hS0 = (1.0 - eta) * st.s0[g] + eta * S[0];
                for (int d = 0; d < 5; ++d) hS1[d] = eta * S[1 + d];
                for (int q = 0; q < 15; ++q) hS2[q] = (1.0 - eta) * st.s2[g * 15 + q] + eta * S[6 + q];
            }
            const double bar0 = act ? hS0 / hW : 0.0;
            const double sum0 = group_sum_fp64<G>(bar0);
            int dead = 0, cholfail = 0;
            if (act) {
                const double mu_in[3] = {mix.mud[3 * g], mix.mud[3 * g + 1], mix.mud[3 * g + 2]};
                const double mux_in[3] = {mix.mux[3 * g], mix.mux[3 * g + 1], mix.mux[3 * g + 2]};
                component_map_update(hS0, hS1, hS2, hW, beta, bar0, o, true, mu_in, mux_in, mix.mud + 3 * g,
                                     mix.mux + 3 * g, mix.cov + 15 * g, st.s0 + g, st.s2 + 15 * g, dead, cholfail);
                mix.pi[g] = (beta * o.prior_q + bar0) / ((double)K * beta * o.prior_q + sum0);
                load_comp(mix, g, cp);
            }
            st_bits |= (wave_any(dead) ? kDeadComponent : 0) | (wave_any(cholfail) ? kCholFailKeptPrev : 0);
            sw = hW;
            ++j;
        }
        if (stop) break;
        if (fresh) {  // one batch step with the accumulated statistics
            bool fin = isfinite(Wb);
            for (int q = 0; q < 21; ++q) fin = fin && isfinite(S[q]);
            if (wave_any(act && !fin)) {
                st_bits |= kBadInput;
                break;
            }
            const double beta = o.prior_mode == 0 ? 1.0 / fmax(Mb, 1.0) : o.prior_scale;
            const double bar0 = act ? S[0] / Wb : 0.0;
            const double sum0 = group_sum_fp64<G>(bar0);
            int dead = 0, cholfail = 0;
            if (act) {
                const double mu_in[3] = {mix.mud[3 * g], mix.mud[3 * g + 1], mix.mud[3 * g + 2]};
                const double mux_in[3] = {mix.mux[3 * g], mix.mux[3 * g + 1], mix.mux[3 * g + 2]};
                component_map_update(S[0], S + 1, S + 6, Wb, beta, bar0, o, true, mu_in, mux_in, mix.mud + 3 * g,
                                     mix.mux + 3 * g, mix.cov + 15 * g, st.s0 + g, st.s2 + 15 * g, dead, cholfail);
                mix.pi[g] = (beta * o.prior_q + bar0) / ((double)K * beta * o.prior_q + sum0);
                load_comp(mix, g, cp);
            }
            st_bits |= (wave_any(dead) ? kDeadComponent : 0) | (wave_any(cholfail) ? kCholFailKeptPrev : 0);
            sw = Wb;
            j = 1;
        }
    }
    if (k == 0) {
        status[c] = st_bits;
        st.sw[c] = sw;
        st.step[c] = j;
    }
}

void launch_stepwise(const int64_t* off, const float* smp, int64_t N, const sdmm_mixtures& mix,
                     const sdmm_em_state& st, const sdmm_fit_opts& opts, int32_t* status, const Layout& L, char* ws,
                     hipStream_t s)
{
    const int C = mix.n_cells;
    const MixPtrs mp{mix.weights, mix.mean_dir, mix.mean_pos, mix.cov};
    const StatePtrs sp{st.s0, st.s2, st.sw, st.step};
    ScopedTimer tm(SDMM_TIMER_STEPWISE, s);
    const int32_t* fl = reinterpret_cast<const int32_t*>(ws + L.flags);
    const int32_t* ctl = reinterpret_cast<const int32_t*>(ws + L.global_ok);
    const DevOpts d = dev_opts(&opts);
    const unsigned blocks = (unsigned)((C + 3) / 4);
    switch (group_for(opts.K)) {
        case 4: stepwise_kernel<4><<<blocks, 256, 0, s>>>(off, N, smp, C, mp, sp, d, opts.iters, fl, ctl, status); break;
        case 8: stepwise_kernel<8><<<blocks, 256, 0, s>>>(off, N, smp, C, mp, sp, d, opts.iters, fl, ctl, status); break;
        case 16:
            stepwise_kernel<16><<<blocks, 256, 0, s>>>(off, N, smp, C, mp, sp, d, opts.iters, fl, ctl, status);
            break;
        case 32:
            stepwise_kernel<32><<<blocks, 256, 0, s>>>(off, N, smp, C, mp, sp, d, opts.iters, fl, ctl, status);
            break;
        default:
            stepwise_kernel<64><<<blocks, 256, 0, s>>>(off, N, smp, C, mp, sp, d, opts.iters, fl, ctl, status);
            break;
    }
}

}  // namespace sdmm
