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
    c.logc = log(pi) - log_det5(c.L) - 2.5 * kLn2Pi;
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
    const double s = sqrt(x * x + yy * yy);  // (x, yy, z) is a unit vector: no overflow
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

// Samples reach the chain through LDS, 64 at a time: lane l loads sample base + l of
// every channel (coalesced; lanes past the end reload the last sample), the loads of the
// next 64 are in flight while the current ones are used, and each step reads its sample
// from LDS by broadcast. No global load is left on the per-sample chain.
__device__ __forceinline__ void stage_fetch(const float* smp, int64_t N, int64_t i, int64_t last, float pre[7])
{
    const int64_t ii = i < last ? i : last;
#pragma unroll
    for (int a = 0; a < 7; ++a) pre[a] = smp[a * N + ii];
}

__device__ __forceinline__ void stage_store(float4 (*stage)[2], int lane, const float pre[7])
{
    __syncthreads();  // the wave is done reading the previous 64
    stage[lane][0] = make_float4(pre[0], pre[1], pre[2], pre[3]);
    stage[lane][1] = make_float4(pre[4], pre[5], pre[6], 0.0f);
    __syncthreads();
}

// Each lane keeps its component in E-step form in LDS, slot by slot with the 64 lanes of
// a slot contiguous (conflict-free), and its factor and carried statistics as rows of
// its own (the update writes a new factor and the new statistics there itself): the E-step copies the
// component into registers for its own span only, and the update, which needs many
// registers of its own, runs without it.
constexpr int kSlotR = 0, kSlotMx = 9, kSlotRd = 12, kSlotLogc = 17, kCompSlots = 18;

__device__ __forceinline__ void comp_put(double (*cs)[64], double* Ls, int lane, const Comp64& c, bool with_L)
{
    for (int q = 0; q < 9; ++q) cs[kSlotR + q][lane] = c.R[q];
    for (int d = 0; d < 3; ++d) cs[kSlotMx + d][lane] = c.mx[d];
    if (with_L)
        for (int q = 0; q < 15; ++q) Ls[q] = c.L[q];
    for (int d = 0; d < 5; ++d) cs[kSlotRd + d][lane] = c.rd[d];
    cs[kSlotLogc][lane] = c.logc;
}

__device__ __forceinline__ void comp_get(double (*cs)[64], const double* Ls, int lane, bool ok, Comp64& c)
{
    for (int q = 0; q < 9; ++q) c.R[q] = cs[kSlotR + q][lane];
    for (int d = 0; d < 3; ++d) c.mx[d] = cs[kSlotMx + d][lane];
    for (int q = 0; q < 15; ++q) c.L[q] = Ls[q];
    for (int d = 0; d < 5; ++d) c.rd[d] = cs[kSlotRd + d][lane];
    c.logc = cs[kSlotLogc][lane];
    c.ok = ok;
}

// The component in E-step form after an update that replaced the covariance of a usable
// component, from what the update produced: the new mean's frame, the new positional
// mean, the diagonal of the update's own factor of the new covariance and its
// reciprocals (the update wrote both to LDS; the factor stays there) and the new weight. This equals load_comp of the stored values:
// from finite statistics the new direction is a unit vector, the positional mean moves
// by a finite weighted mean, and the weight's denominator is at least this component's
// bar0, above the dead threshold, so load_comp's finiteness checks would pass.
__device__ __forceinline__ void refresh_comp(Comp64& c, const double mu[3], const double mx[3], const double* L,
                                             double pi)
{
    c.ok = true;
    frame64(mu, c.R);
    for (int d = 0; d < 3; ++d) c.mx[d] = mx[d];
    for (int d = 0; d < 5; ++d) {
        c.L[tri(d, d)] = L[tri(d, d)];
        c.rd[d] = L[15 + d];
    }
    set_log_constant(c, pi);
}

// One wave (= one work group) per cell.
template <int G>
__global__ __launch_bounds__(64) void stepwise_kernel(const int64_t* __restrict__ off, int64_t N,
                                                      const float* __restrict__ smp, int C, MixPtrs mix,
                                                      StatePtrs st, DevOpts o, int iters,
                                                      const int32_t* __restrict__ flags,
                                                      const int32_t* __restrict__ control,
                                                      int32_t* __restrict__ status)
{
    __shared__ float4 stage[64][2];
    __shared__ double comp[kCompSlots][64];
    __shared__ double stat[64][17];  // per lane s0, then s2, one pad (row stride of 34 dwords)
    __shared__ double eta_s[64];    // step sizes of the next 64 sample counters
    __shared__ double Lsh[64][21];  // factor, reciprocals of its diagonal, one pad (row stride
                                    // of 42 dwords: the 64 lanes start on 32 distinct banks)
    const int c = blockIdx.x;
    if (c >= C) return;
    const int K = o.K;
    const int k = threadIdx.x;
    const bool act = k < K;
    const int64_t g = (int64_t)c * K + (act ? k : 0);
    const bool jac = (o.flags & SDMM_FLAG_ESTEP_JACOBIAN) != 0;
    int st_bits = 0;
    const int64_t i0 = off[c], i1 = off[c + 1];
    const bool range_ok = control[0] && !(flags[c] & kFlagBadRange);
    int j = st.step[c];
    double sw = st.sw[c];
    for (int q = 0; q < 16; ++q) stat[k][q] = q == 0 ? st.s0[g] : st.s2[g * 15 + q - 1];
    bool cok;
    {
        Comp64 cp;
        load_comp(mix, g, cp);
        comp_put(comp, Lsh[k], k, cp, true);
        cok = cp.ok;
    }
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
        const bool badp = wave_any(act && !cok);
        int gate = 0;
        if (any_bad) gate = kBadInput;
        else if (badp) gate = kBadParams;
        else if (Mt < (double)o.min_samples) gate = kSkippedFew;
        else if (!(Wt > 0.0)) gate = kSkippedZeroW;
        if (gate) {
            st_bits |= gate;
            break;
        }
        // (the gate passed, so i0 < i1 <= N)
        float pre[7];
        stage_fetch(smp, N, i0 + k, i1 - 1, pre);
        if (j == 0) {
            // a fresh cell: the statistics of the whole batch in sample order, then one
            // batch step
            double S[21];
            double Wb = 0.0, Mb = 0.0;
            for (int q = 0; q < 21; ++q) S[q] = 0.0;
            Comp64 cp;
            comp_get(comp, Lsh[k], k, cok, cp);
            for (int64_t base = i0; base < i1; base += 64) {
                stage_store(stage, k, pre);
                if (base + 64 < i1) stage_fetch(smp, N, base + 64 + k, i1 - 1, pre);
                const int n = (int)(i1 - base < 64 ? i1 - base : 64);
                for (int t = 0; t < n; ++t) {
                    const float4 a = stage[t][0], b = stage[t][1];
                    const double wi = (double)b.z;
                    Wb += wi;
                    Mb += wi > 0.0 ? 1.0 : 0.0;
                    const double w[3] = {(double)a.x, (double)a.y, (double)a.z};
                    const double p[3] = {(double)a.w, (double)b.x, (double)b.y};
                    double y[5];
                    double l = comp_log_density(cp, w, p, jac, y);
                    if (!act) l = -INFINITY;
                    const double lmax = group_max_fp64<G>(l);
                    const double e = act ? exp(l - lmax) : 0.0;
                    const double den = group_sum_fp64<G>(e);
                    const double wr = act ? wi * (e / den) : 0.0;
                    S[0] += wr;
                    for (int d = 0; d < 5; ++d) {
                        S[1 + d] += wr * y[d];
                        for (int f = 0; f <= d; ++f) S[6 + tri(d, f)] += wr * y[d] * y[f];
                    }
                }
            }
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
                                     mix.mux + 3 * g, mix.cov + 15 * g, &stat[k][0], &stat[k][1], dead, cholfail);
                mix.pi[g] = (beta * o.prior_q + bar0) / ((double)K * beta * o.prior_q + sum0);
                load_comp(mix, g, cp);
                comp_put(comp, Lsh[k], k, cp, true);
                cok = cp.ok;
            }
            st_bits |= (wave_any(dead) ? kDeadComponent : 0) | (wave_any(cholfail) ? kCholFailKeptPrev : 0);
            sw = Wb;
            j = 1;
            continue;
        }
        // every sample with positive weight is a mini-batch of one
        bool stop = false;
        for (int64_t base = i0; base < i1 && !stop; base += 64) {
            // the 64 samples, and the Robbins-Monro step sizes of the sample counters they
            // can reach (the counter rises by at most one per sample): one per lane
            const int jb = j;
            __syncthreads();
            stage[k][0] = make_float4(pre[0], pre[1], pre[2], pre[3]);
            stage[k][1] = make_float4(pre[4], pre[5], pre[6], 0.0f);
            eta_s[k] = rm_eta(o, jb + k);
            __syncthreads();
            if (base + 64 < i1) stage_fetch(smp, N, base + 64 + k, i1 - 1, pre);
            const int n = (int)(i1 - base < 64 ? i1 - base : 64);
            for (int t = 0; t < n; ++t) {
                const float4 a = stage[t][0], b = stage[t][1];
                const double wi = (double)b.z;
                if (!(wi > 0.0)) continue;
                const double eta = eta_s[j - jb];
                double y[5], l, mu[3], mx[3];
                {
                    Comp64 cp;
                    comp_get(comp, Lsh[k], k, cok, cp);
                    const double w[3] = {(double)a.x, (double)a.y, (double)a.z};
                    const double p[3] = {(double)a.w, (double)b.x, (double)b.y};
                    l = comp_log_density(cp, w, p, jac, y);
                    // the current means of a usable component (its frame's last row is its mean)
                    for (int d = 0; d < 3; ++d) {
                        mu[d] = cp.R[6 + d];
                        mx[d] = cp.mx[d];
                    }
                }
                if (!act) l = -INFINITY;
                // the log-sum-exp over the component lanes (the first G lanes hold the
                // cell's components; the other groups of G lanes hold only inactive lanes)
                const double lmax = group_max_fp64<G>(l);
                const double e = act ? exp(l - lmax) : 0.0;
                const double den = group_sum_fp64<G>(e);
                const double wr = act ? wi * (e / den) : 0.0;
                double S[21];
                S[0] = wr;
                for (int d = 0; d < 5; ++d) {
                    S[1 + d] = wr * y[d];
                    for (int f = 0; f <= d; ++f) S[6 + tri(d, f)] = wr * y[d] * y[f];
                }
                bool fin = isfinite(wi);
                for (int q = 0; q < 21; ++q) fin = fin && isfinite(S[q]);
                if (wave_any(act && !fin)) {
                    st_bits |= kBadInput;
                    stop = true;
                    break;
                }
                const double beta = o.prior_mode == 0 ? eta : o.prior_scale;
                const double hW = (1.0 - eta) * sw + eta * wi;
                double hS0 = 0.0, hS1[5], hS2[15];
                if (act) {
                    hS0 = (1.0 - eta) * stat[k][0] + eta * S[0];
                    for (int d = 0; d < 5; ++d) hS1[d] = eta * S[1 + d];
                    for (int q = 0; q < 15; ++q) hS2[q] = (1.0 - eta) * stat[k][1 + q] + eta * S[6 + q];
                }
                const double bar0 = act ? hS0 / hW : 0.0;
                const double sum0 = group_sum_fp64<G>(bar0);
                int dead = 0, cholfail = 0;
                if (act) {
                    if (!cok)  // an unusable component's means come from memory
                        for (int d = 0; d < 3; ++d) {
                            mu[d] = mix.mud[3 * g + d];
                            mx[d] = mix.mux[3 * g + d];
                        }
                    const double mu_in[3] = {mu[0], mu[1], mu[2]};
                    const double mux_in[3] = {mx[0], mx[1], mx[2]};
                    component_map_update(hS0, hS1, hS2, hW, beta, bar0, o, true, mu_in, mux_in, mu, mx,
                                         mix.cov + 15 * g, &stat[k][0], &stat[k][1], dead, cholfail, Lsh[k]);
                    const double pin = (beta * o.prior_q + bar0) / ((double)K * beta * o.prior_q + sum0);
                    mix.pi[g] = pin;
                    for (int d = 0; d < 3; ++d) {
                        mix.mud[3 * g + d] = mu[d];
                        mix.mux[3 * g + d] = mx[d];
                    }
                    // a dead component, a kept covariance or an unusable one reloads
                    Comp64 cn;
                    const bool rebuilt = cok && !dead && !cholfail;
                    if (rebuilt) refresh_comp(cn, mu, mx, Lsh[k], pin);
                    else load_comp(mix, g, cn);
                    comp_put(comp, Lsh[k], k, cn, !rebuilt);
                    cok = cn.ok;
                }
                st_bits |= (wave_any(dead) ? kDeadComponent : 0) | (wave_any(cholfail) ? kCholFailKeptPrev : 0);
                sw = hW;
                ++j;
            }
        }
        if (stop) break;
    }
    if (act) {
        st.s0[g] = stat[k][0];
        for (int q = 0; q < 15; ++q) st.s2[g * 15 + q] = stat[k][1 + q];
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
    const unsigned blocks = (unsigned)C;
    switch (group_for(opts.K)) {
        case 4: stepwise_kernel<4><<<blocks, 64, 0, s>>>(off, N, smp, C, mp, sp, d, opts.iters, fl, ctl, status); break;
        case 8: stepwise_kernel<8><<<blocks, 64, 0, s>>>(off, N, smp, C, mp, sp, d, opts.iters, fl, ctl, status); break;
        case 16:
            stepwise_kernel<16><<<blocks, 64, 0, s>>>(off, N, smp, C, mp, sp, d, opts.iters, fl, ctl, status);
            break;
        case 32:
            stepwise_kernel<32><<<blocks, 64, 0, s>>>(off, N, smp, C, mp, sp, d, opts.iters, fl, ctl, status);
            break;
        default:
            stepwise_kernel<64><<<blocks, 64, 0, s>>>(off, N, smp, C, mp, sp, d, opts.iters, fl, ctl, status);
            break;
    }
}

}  // namespace sdmm
