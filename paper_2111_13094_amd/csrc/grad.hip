// grad.hip -- value and gradient of the weighted penalised log-likelihood
//   F = sum_i (w_i / W) log sum_k pi_k N5(y_ik; 0, Sigma_k)
//       + sum_k [beta q log pi_k - (beta a / 2) log det Sigma_k - (beta / 2) tr(B Sigma_k^-1)],
// the objective whose maximiser is the MAP update of Sec. 4.3 of Dodik et al. (Dirichlet
// prior on the weights, inverse-Wishart prior on the covariances, none on the means).
//
// One pass over the samples (the E-step pass with extra accumulators) gives, per
// component and about the current means, S0, S1, S2, sum w r (d nu / d delta)^T
// [Sigma^-1 y]_nu, and per cell sum w log p. A per-cell FP64 assembly then forms
//   dF/dalpha_k = S0_k/W + beta q - pi_k (sum_j S0_j/W + K beta q)        (pi = softmax alpha)
//   dF/dmu_x_k  = [Sigma_k^-1 S1_k / W]_x
//   dF/dL_k     = tril(2 G_k L_k),  G_k = 1/2 Sigma^-1 (S2/W + beta B) Sigma^-1
//                                        - 1/2 (S0/W + beta a) Sigma^-1
//   dF/ddelta_k = -(1/W) sum_i w_i r_ik (d nu_ik / d delta)^T [Sigma_k^-1 y_ik]_nu
#include "common.hpp"
#include "estep.hpp"
#include "timing.hpp"

namespace sdmm {

__device__ __forceinline__ double gsum(double v, int GM)
{
    for (int o = 1; o < GM; o <<= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ int gor(int v, int GM)
{
    for (int o = 1; o < GM; o <<= 1) v |= __shfl_xor(v, o);
    return v;
}

// one wave per cell: all lanes sum the cell's records, lane k = component k (k < G)
template <int G>
__global__ __launch_bounds__(256) void grad_assemble_kernel(const int64_t* __restrict__ off, int64_t N, int C,
                                                            int ps, const double* __restrict__ records, int PS,
                                                            const int32_t* __restrict__ flags,
                                                            const int32_t* __restrict__ global_ok,
                                                            const float* __restrict__ mirror, MixPtrs mix, DevOpts o,
                                                            double* __restrict__ F_out, double* __restrict__ g_alpha,
                                                            double* __restrict__ g_mux, double* __restrict__ g_delta,
                                                            double* __restrict__ g_L, int32_t* __restrict__ status)
{
    constexpr int NS = ChunkLayout<true>::kNStat;
    constexpr int GM = G;
    const int K = o.K;
    const int c0i = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const bool wave_ok = c0i < C;
    const int c = wave_ok ? c0i : 0;
    const bool cell_ok = wave_ok && lane < G;
    const int k = lane;
    const bool act = cell_ok && k < K;
    const int kk = k < K ? k : 0;

    double S[NS], X[4];
    int64_t first = 0, n_items = 0;
    const bool have = wave_ok && cell_items(off, N, c, ps, first, n_items);
    const int lv = *global_ok ? tree_levels_done(global_ok) : 0;  // top leaders of the record tree
    sum_cell_records<G, NS, 4>(records, first, have ? n_items : 0, PS, kTreeLog2R * lv, S, X);
    const double W = X[0], Mc = X[1], negs = X[2], LL = X[3];
    int fin = isfinite(W) && isfinite(LL);
    for (int s = 0; s < NS; ++s) fin &= isfinite(S[s]) ? 1 : 0;
    const int notfin = gor(act && !fin ? 1 : 0, GM) | (!(isfinite(W) && isfinite(LL)) ? 1 : 0);
    int gate = 0;
    if (cell_ok) {
        const int fl = flags[c];
        if (negs > 0.0 || notfin || (fl & kFlagBadRange) || !*global_ok) gate = kBadInput;
        else if (fl & kBadParams) gate = kBadParams;
        else if (Mc < (double)o.min_samples) gate = kSkippedFew;
        else if (!(W > 0.0)) gate = kSkippedZeroW;
    }
    const int64_t g = (int64_t)c * K + kk;
    if (gate) {
        if (act) {
            g_alpha[g] = 0.0;
            for (int d = 0; d < 3; ++d) g_mux[3 * g + d] = 0.0;
            for (int d = 0; d < 2; ++d) g_delta[2 * g + d] = 0.0;
            for (int q = 0; q < 15; ++q) g_L[15 * g + q] = 0.0;
        }
        if (cell_ok && k == 0) {
            F_out[c] = 0.0;
            status[c] = gate;
        }
        return;
    }
    const double beta = o.prior_scale;
    const double b0 = act ? S[0] / W : 0.0;
    const double sum0 = gsum(b0, GM);
    double Fk = 0.0;
    if (act) {
        const double pik = mix.pi[g];
        g_alpha[g] = b0 + beta * o.prior_q - pik * (sum0 + (double)K * beta * o.prior_q);
        double L[15], Li[15];
        chol64<5>(mix.cov + 15 * g, L);
        tri_inv64<5>(L, Li);
        double Si[5][5];  // Sigma^-1 = Li^T Li
        for (int d = 0; d < 5; ++d)
            for (int e = 0; e < 5; ++e) {
                double s = 0.0;
                for (int f = (d > e ? d : e); f < 5; ++f) s += Li[tri(f, d)] * Li[tri(f, e)];
                Si[d][e] = s;
            }
        for (int d = 0; d < 3; ++d) {
            double s = 0.0;
            for (int e = 0; e < 5; ++e) s += Si[2 + d][e] * S[1 + e] / W;
            g_mux[3 * g + d] = s;
        }
        double A[5][5];
        for (int d = 0; d < 5; ++d)
            for (int e = 0; e < 5; ++e) {
                const int dd = d > e ? d : e, ee = d > e ? e : d;
                A[d][e] = S[6 + tri(dd, ee)] / W + (d == e ? beta * o.prior_b[d] : 0.0);
            }
        double SA[5][5], Gm[5][5];
        for (int d = 0; d < 5; ++d)
            for (int e = 0; e < 5; ++e) {
                double s = 0.0;
                for (int f = 0; f < 5; ++f) s += Si[d][f] * A[f][e];
                SA[d][e] = s;
            }
        for (int d = 0; d < 5; ++d)
            for (int e = 0; e < 5; ++e) {
                double s = 0.0;
                for (int f = 0; f < 5; ++f) s += SA[d][f] * Si[f][e];
                Gm[d][e] = 0.5 * s - 0.5 * (b0 + beta * o.prior_a) * Si[d][e];
            }
        for (int d = 0; d < 5; ++d)
            for (int e = 0; e <= d; ++e) {
                double s = 0.0;
                for (int p = e; p < 5; ++p) s += Gm[d][p] * L[tri(p, e)];
                g_L[15 * g + tri(d, e)] = 2.0 * s;
            }
        // the device pass accumulated (log2(e)/2) Sigma^-1 y
        const double unscale = 1.0 / (0.5 * kLog2e);
        g_delta[2 * g] = -S[21] / W * unscale;
        g_delta[2 * g + 1] = -S[22] / W * unscale;
        double logdet = 0.0;
        for (int d = 0; d < 5; ++d) logdet += 2.0 * log(L[tri(d, d)]);
        double tr = 0.0;
        for (int d = 0; d < 5; ++d) tr += o.prior_b[d] * Si[d][d];
        Fk = beta * o.prior_q * log(pik) - 0.5 * beta * o.prior_a * logdet - 0.5 * beta * tr;
    }
    Fk = gsum(Fk, GM);
    if (cell_ok && k == 0) {
        // the pass accumulated shifted log2 densities; add the cell's shift back
        const double shift = (double)mirror[(int64_t)c * K * kMirror + kMirShift];
        F_out[c] = (LL + shift * W) / kLog2e / W + Fk;
        status[c] = 0;
    }
}

}  // namespace sdmm

using namespace sdmm;

extern "C" int sdmm_fit_grad(const int64_t* cell_offsets, const float* samples, int64_t n_samples,
                             const sdmm_mixtures* mix, const sdmm_fit_opts* opts, double* F_out, double* g_alpha,
                             double* g_mu_pos, double* g_delta, double* g_L, int32_t* cell_status, void* workspace,
                             size_t workspace_bytes, void* stream)
{
    int rc = validate_fit_args(cell_offsets, samples, n_samples, mix, opts, cell_status, workspace, workspace_bytes);
    if (rc) return rc;
    if (!F_out || !g_alpha || !g_mu_pos || !g_delta || !g_L) return SDMM_EINVAL;
    if (opts->flags & SDMM_FLAG_ESTEP_JACOBIAN) return SDMM_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int C = mix->n_cells, K = mix->K;
    const Layout L = layout_for(C, K, n_samples, opts);
    char* ws = reinterpret_cast<char*>(workspace);
    mark_mirrors(workspace, *mix, false);  // the setup below rewrites the workspace
    launch_setup(cell_offsets, n_samples, *mix, cell_status, ws, L, s, true);
    {
        ScopedTimer tm(SDMM_TIMER_GRAD, s);
        // as in the fit: a work item that fits one block of the compensated sums runs the
        // plain-sum pass, bit for bit the same with fewer registers
        const int G = group_for(K);
        const bool one_block = (L.P / (64 / G)) <= kFoldEvery;
        const EstepFn pass = (opts->flags & SDMM_FLAG_FP64_SUMS)
                                 ? adj64_function(G)
                                 : estep_function(G, one_block ? kAccPlain : kAccTwoSum, false, true);
        launch_estep(pass, samples, n_samples, cell_offsets, C,
                     K, L, 0, (int64_t)C + L.W, L.ps_grad, ws, s);
    }
    launch_tree(kTreeGrad, cell_offsets, n_samples, C, K, L, -1, 0, 0, ws, s, false);
    const MixPtrs mp{mix->weights, mix->mean_dir, mix->mean_pos, mix->cov};
    auto asm_fn = grad_assemble_kernel<16>;
    switch (group_for(K)) {
        case 4: asm_fn = grad_assemble_kernel<4>; break;
        case 8: asm_fn = grad_assemble_kernel<8>; break;
        case 16: asm_fn = grad_assemble_kernel<16>; break;
        case 32: asm_fn = grad_assemble_kernel<32>; break;
        default: asm_fn = grad_assemble_kernel<64>; break;
    }
    hipLaunchKernelGGL(asm_fn, dim3((C + 3) / 4), dim3(256), 0, s, cell_offsets, n_samples, C, L.ps,
                       reinterpret_cast<const double*>(ws + L.records), L.ps_grad,
                       reinterpret_cast<const int32_t*>(ws + L.flags),
                       reinterpret_cast<const int32_t*>(ws + L.global_ok), reinterpret_cast<const float*>(ws + L.mirror),
                       mp, dev_opts(opts), F_out, g_alpha, g_mu_pos, g_delta, g_L, cell_status);
    return check(hipGetLastError());
}
