// grad.hip -- value and gradient of the weighted penalised log-likelihood
//   F = sum_i (w_i / W) log sum_k pi_k N5(y_ik; 0, Sigma_k)
//       + sum_k [beta q log pi_k - (beta a / 2) log det Sigma_k - (beta / 2) tr(B Sigma_k^-1)],
// the objective whose maximiser is the MAP update of Sec. 4.3 of Dodik et al. (Dirichlet
// prior on the weights, inverse-Wishart prior on the covariances, none on the means).
//
// One pass over the samples (the E-step pass with two extra accumulators) gives, per
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

template <int G>
__global__ __launch_bounds__(256) void grad_estep_kernel(const float* __restrict__ smp, int64_t N,
                                                         const int64_t* __restrict__ off,
                                                         const int32_t* __restrict__ chunk_cell,
                                                         const int32_t* __restrict__ chunk_start,
                                                         const int32_t* __restrict__ n_total,
                                                         const float* __restrict__ mirror, int K, int64_t chunk,
                                                         int PS, double* __restrict__ partial)
{
    extern __shared__ double lds[];
    const int t = blockIdx.x;
    if (t >= *n_total) return;
    const int c = chunk_cell[t];
    int64_t c0, c1;
    cell_range(off, c, N, c0, c1);
    const int64_t cs = chunk_size_for(c1 - c0, chunk);
    const int64_t s0 = min(c1, c0 + (int64_t)(t - chunk_start[c]) * cs);
    const int64_t s1 = min(c1, s0 + cs);
    estep_chunk<G, kAccTwoSum, false, true>(smp, N, s0, s1, mirror + (int64_t)c * K * kMirror, K,
                                            partial + (int64_t)t * PS, lds);
}

__global__ __launch_bounds__(64) void grad_assemble_kernel(const int32_t* __restrict__ chunk_start,
                                                           const double* __restrict__ partial, int PS,
                                                           const int32_t* __restrict__ flags, MixPtrs mix, DevOpts o,
                                                           double* __restrict__ F_out, double* __restrict__ g_alpha,
                                                           double* __restrict__ g_mux, double* __restrict__ g_delta,
                                                           double* __restrict__ g_L, int32_t* __restrict__ status)
{
    constexpr int NS = ChunkLayout<true>::kNStat;
    __shared__ double red[NS * kMaxK + 4];
    const int c = blockIdx.x;
    const int K = o.K;
    const int lane = threadIdx.x & 63;
    const int t0 = chunk_start[c], t1 = chunk_start[c + 1];
    const int nv = NS * K + 4;
    for (int v = lane; v < nv; v += 64) {
        double s = 0.0;
        for (int t = t0; t < t1; ++t) s += partial[(int64_t)t * PS + v];
        red[v] = s;
    }
    __syncthreads();
    const double W = red[NS * K], Mc = red[NS * K + 1], negs = red[NS * K + 2], LL = red[NS * K + 3];
    bool fin = isfinite(W) && isfinite(LL);
    for (int v = lane; v < NS * K; v += 64) fin = fin && isfinite(red[v]);
    fin = __all(fin);
    int gate = 0;
    if (negs > 0.0 || !fin || (flags[c] & kFlagBadRange)) gate = kBadInput;
    else if (flags[c] & kBadParams) gate = kBadParams;
    else if (Mc < (double)o.min_samples) gate = kSkippedFew;
    else if (!(W > 0.0)) gate = kSkippedZeroW;
    const int k = lane;
    const bool act = k < K;
    const int64_t g = (int64_t)c * K + (act ? k : 0);
    if (gate) {
        if (act) {
            g_alpha[g] = 0.0;
            for (int d = 0; d < 3; ++d) g_mux[3 * g + d] = 0.0;
            for (int d = 0; d < 2; ++d) g_delta[2 * g + d] = 0.0;
            for (int q = 0; q < 15; ++q) g_L[15 * g + q] = 0.0;
        }
        if (lane == 0) {
            F_out[c] = 0.0;
            status[c] = gate;
        }
        return;
    }
    const double beta = o.prior_scale;
    const double b0 = act ? red[k] / W : 0.0;
    double sum0 = b0;
    for (int ofs = 1; ofs < 64; ofs <<= 1) sum0 += __shfl_xor(sum0, ofs);
    double Fk = 0.0;
    if (act) {
        const double pik = mix.pi[g];
        g_alpha[g] = b0 + beta * o.prior_q - pik * (sum0 + (double)K * beta * o.prior_q);
        double L[15], Li[15];
        chol64<5>(mix.cov + 15 * g, L);
        tri_inv64<5>(L, Li);
        // Sigma^-1 = Li^T Li (dense)
        double Si[5][5];
        for (int d = 0; d < 5; ++d)
            for (int e = 0; e < 5; ++e) {
                double s = 0.0;
                for (int f = (d > e ? d : e); f < 5; ++f) s += Li[tri(f, d)] * Li[tri(f, e)];
                Si[d][e] = s;
            }
        for (int d = 0; d < 3; ++d) {
            double s = 0.0;
            for (int e = 0; e < 5; ++e) s += Si[2 + d][e] * red[(1 + e) * K + k] / W;
            g_mux[3 * g + d] = s;
        }
        double A[5][5];
        for (int d = 0; d < 5; ++d)
            for (int e = 0; e < 5; ++e) {
                const int dd = d > e ? d : e, ee = d > e ? e : d;
                A[d][e] = red[(6 + tri(dd, ee)) * K + k] / W + (d == e ? beta * o.prior_b[d] : 0.0);
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
        g_delta[2 * g] = -red[21 * K + k] / W * unscale;
        g_delta[2 * g + 1] = -red[22 * K + k] / W * unscale;
        double logdet = 0.0;
        for (int d = 0; d < 5; ++d) logdet += 2.0 * log(L[tri(d, d)]);
        double tr = 0.0;
        for (int d = 0; d < 5; ++d) tr += o.prior_b[d] * Si[d][d];
        Fk = beta * o.prior_q * log(pik) - 0.5 * beta * o.prior_a * logdet - 0.5 * beta * tr;
    }
    for (int ofs = 1; ofs < 64; ofs <<= 1) Fk += __shfl_xor(Fk, ofs);
    if (lane == 0) {
        F_out[c] = LL / W + Fk;
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
    const int64_t chunk = default_chunk(opts);
    const int waves = default_waves(opts);
    const Layout L = layout_for(C, K, n_samples, chunk);
    char* ws = reinterpret_cast<char*>(workspace);
    launch_plan_prepare(cell_offsets, n_samples, *mix, chunk, cell_status, ws, L, s);
    const float* mirror = reinterpret_cast<const float*>(ws + L.mirror);
    const int32_t* flags = reinterpret_cast<const int32_t*>(ws + L.flags);
    const int32_t* cstart = reinterpret_cast<const int32_t*>(ws + L.chunk_start);
    const int32_t* ccell = reinterpret_cast<const int32_t*>(ws + L.chunk_cell);
    const int32_t* ntot = reinterpret_cast<const int32_t*>(ws + L.n_total);
    double* partial = reinterpret_cast<double*>(ws + L.partial);
    const int G = group_for(K);
    const size_t lds = (size_t)waves * ChunkLayout<true>::kNRed * G * sizeof(double);
    const dim3 grid((unsigned)L.tmax), block(waves * 64);
    ScopedTimer tm(SDMM_TIMER_GRAD, s);
    switch (G) {
        case 4: grad_estep_kernel<4><<<grid, block, lds, s>>>(samples, n_samples, cell_offsets, ccell, cstart, ntot, mirror, K, chunk, L.ps_grad, partial); break;
        case 8: grad_estep_kernel<8><<<grid, block, lds, s>>>(samples, n_samples, cell_offsets, ccell, cstart, ntot, mirror, K, chunk, L.ps_grad, partial); break;
        case 16: grad_estep_kernel<16><<<grid, block, lds, s>>>(samples, n_samples, cell_offsets, ccell, cstart, ntot, mirror, K, chunk, L.ps_grad, partial); break;
        case 32: grad_estep_kernel<32><<<grid, block, lds, s>>>(samples, n_samples, cell_offsets, ccell, cstart, ntot, mirror, K, chunk, L.ps_grad, partial); break;
        default: grad_estep_kernel<64><<<grid, block, lds, s>>>(samples, n_samples, cell_offsets, ccell, cstart, ntot, mirror, K, chunk, L.ps_grad, partial); break;
    }
    const MixPtrs mp{mix->weights, mix->mean_dir, mix->mean_pos, mix->cov};
    grad_assemble_kernel<<<C, 64, 0, s>>>(cstart, partial, L.ps_grad, flags, mp, dev_opts(opts), F_out, g_alpha,
                                          g_mu_pos, g_delta, g_L, cell_status);
    return check(hipGetLastError());
}
