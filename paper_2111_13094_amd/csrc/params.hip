// params.hip -- the unconstrained parameterisation used for gradient-based refinement of
// the fitted mixtures, and the pull-back of the adjoint's gradients onto it.
//
//   pi_k     = softmax(alpha)_k within the cell
//   mu_dir_k = exp_{mu0_k}(delta_k)        (exp map of Sec. 3.1, frame of mu0_k as in the fit)
//   mu_pos_k = mu_pos_k
//   Sigma_k  = L_k L_k^T                    (packed lower-triangular L_k)
//
// sdmm_fit_grad differentiates about the current directional mean, i.e. with respect to
// delta' in exp_{mu_dir}(delta'). With mu_dir = exp_{mu0}(delta), a change eps of delta
// moves the point to delta' = log_{mu_dir}(exp_{mu0}(delta + eps)) = J eps + O(eps^2), J the
// first-order transfer Jacobian of Sec. 3.4 evaluated at nu = delta; so dF/ddelta = J^T dF/ddelta'.
// sdmm_fit_grad also factors Sigma again; its Cholesky factor is L D with D = diag(sign L_ee),
// so dF/dL = tril(2 G L) = tril(2 G L D) D, a sign flip of the columns with negative pivots.
#include "common.hpp"

namespace sdmm {

__global__ __launch_bounds__(256) void mixture_from_params_kernel(int C, int K, const double* __restrict__ alpha,
                                                                  const double* __restrict__ mu0,
                                                                  const double* __restrict__ delta,
                                                                  const double* __restrict__ mu_pos,
                                                                  const double* __restrict__ L, MixPtrs out,
                                                                  double* __restrict__ jac, int GM)
{
    const int per_block = blockDim.x / GM;
    const int c = blockIdx.x * per_block + threadIdx.x / GM;
    const int k = threadIdx.x % GM;
    const bool act = c < C && k < K;
    const int64_t g = (int64_t)(act ? c : 0) * K + (act ? k : 0);
    // softmax over the cell's logits, FP64
    double a = act ? alpha[g] : -INFINITY;
    double amax = a;
    for (int o = 1; o < GM; o <<= 1) amax = fmax(amax, __shfl_xor(amax, o));
    double e = act ? exp(a - amax) : 0.0;
    double es = e;
    for (int o = 1; o < GM; o <<= 1) es += __shfl_xor(es, o);
    if (!act) return;
    out.pi[g] = e / es;
    double m0[3] = {mu0[3 * g], mu0[3 * g + 1], mu0[3 * g + 2]};
    const double n0 = 1.0 / sqrt(m0[0] * m0[0] + m0[1] * m0[1] + m0[2] * m0[2]);
    for (int j = 0; j < 3; ++j) m0[j] *= n0;
    double Ro[9], Rn[9], w[3];
    frame64(m0, Ro);
    const double d0 = delta[2 * g], d1 = delta[2 * g + 1];
    const TangentRadius64 tr = tangent_radius64(d0, d1);
    exp_map64(Ro, d0, d1, tr, w);
    const double nw = 1.0 / sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    for (int j = 0; j < 3; ++j) {
        w[j] *= nw;
        out.mud[3 * g + j] = w[j];
        out.mux[3 * g + j] = mu_pos[3 * g + j];
    }
    if (jac) {
        frame64(w, Rn);
        double J[4];
        transfer_jac64(Ro, Rn, d0, d1, tr, J);
        for (int q = 0; q < 4; ++q) jac[4 * g + q] = J[q];
    }
    const double* l = L + 15 * g;
    for (int d = 0; d < 5; ++d)
        for (int f = 0; f <= d; ++f) {
            double s = 0.0;
            for (int p = 0; p <= f; ++p) s += l[tri(d, p)] * l[tri(f, p)];
            out.cov[15 * g + tri(d, f)] = s;
        }
}

__global__ __launch_bounds__(256) void grad_to_params_kernel(int64_t n, const double* __restrict__ L,
                                                             const double* __restrict__ jac,
                                                             double* __restrict__ g_delta, double* __restrict__ g_L)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const double* J = jac + 4 * g;
    const double a = g_delta[2 * g], b = g_delta[2 * g + 1];
    g_delta[2 * g] = J[0] * a + J[2] * b;
    g_delta[2 * g + 1] = J[1] * a + J[3] * b;
    for (int e = 0; e < 5; ++e)
        if (L[15 * g + tri(e, e)] < 0.0)
            for (int d = e; d < 5; ++d) g_L[15 * g + tri(d, e)] = -g_L[15 * g + tri(d, e)];
}

// alpha = log pi, L = chol(Sigma); lanes of cells whose Sigma is not SPD or pi not positive
// get L = 0 / alpha = -inf, and the cell a BAD_PARAMS status
__global__ __launch_bounds__(256) void params_from_mixture_kernel(int C, int K, MixPtrs mix,
                                                                  double* __restrict__ alpha,
                                                                  double* __restrict__ L,
                                                                  int32_t* __restrict__ status, int GM)
{
    const int per_block = blockDim.x / GM;
    const int c = blockIdx.x * per_block + threadIdx.x / GM;
    const int k = threadIdx.x % GM;
    const bool act = c < C && k < K;
    int bad = 0;
    if (act) {
        const int64_t g = (int64_t)c * K + k;
        const double p = mix.pi[g];
        alpha[g] = p > 0.0 ? log(p) : -INFINITY;
        double l[15];
        const bool ok = chol64<5>(mix.cov + 15 * g, l);
        for (int q = 0; q < 15; ++q) L[15 * g + q] = ok ? l[q] : 0.0;
        bad = !ok || !(p > 0.0) || !isfinite(p);
    }
    for (int o = 1; o < GM; o <<= 1) bad |= __shfl_xor(bad, o);
    if (c < C && k == 0 && status) status[c] = bad ? kBadParams : 0;
}

}  // namespace sdmm

using namespace sdmm;

extern "C" int sdmm_params_from_mixture(const sdmm_mixtures* mix, double* alpha, double* L, int32_t* cell_status,
                                        void* stream)
{
    if (!mix || mix->n_cells < 0 || mix->K < 1 || mix->K > kMaxK) return SDMM_EINVAL;
    if (mix->n_cells == 0) return SDMM_OK;
    if (!alpha || !L || !mix->weights || !mix->cov) return SDMM_EINVAL;
    const int GM = group_pow2(mix->K);
    const int per_block = 256 / GM;
    const MixPtrs mp{mix->weights, mix->mean_dir, mix->mean_pos, mix->cov};
    params_from_mixture_kernel<<<(mix->n_cells + per_block - 1) / per_block, 256, 0,
                                 reinterpret_cast<hipStream_t>(stream)>>>(mix->n_cells, mix->K, mp, alpha, L,
                                                                          cell_status, GM);
    return check(hipGetLastError());
}

extern "C" int sdmm_mixture_from_params(int32_t n_cells, int32_t K, const double* alpha, const double* mu_dir0,
                                        const double* delta, const double* mu_pos, const double* L,
                                        const sdmm_mixtures* out, double* jac_out, void* stream)
{
    if (n_cells < 0 || K < 1 || K > kMaxK || !out || out->n_cells != n_cells || out->K != K) return SDMM_EINVAL;
    if (n_cells == 0) return SDMM_OK;
    if (!alpha || !mu_dir0 || !delta || !mu_pos || !L || !out->weights || !out->mean_dir || !out->mean_pos ||
        !out->cov)
        return SDMM_EINVAL;
    const int GM = group_pow2(K);
    const int per_block = 256 / GM;
    const MixPtrs mp{out->weights, out->mean_dir, out->mean_pos, out->cov};
    mixture_from_params_kernel<<<(n_cells + per_block - 1) / per_block, 256, 0,
                                 reinterpret_cast<hipStream_t>(stream)>>>(n_cells, K, alpha, mu_dir0, delta, mu_pos,
                                                                          L, mp, jac_out, GM);
    return check(hipGetLastError());
}

extern "C" int sdmm_grad_to_params(int32_t n_cells, int32_t K, const double* L, const double* jac, double* g_delta,
                                   double* g_L, void* stream)
{
    if (n_cells < 0 || K < 1 || K > kMaxK) return SDMM_EINVAL;
    const int64_t n = (int64_t)n_cells * K;
    if (n == 0) return SDMM_OK;
    if (!L || !jac || !g_delta || !g_L) return SDMM_EINVAL;
    grad_to_params_kernel<<<(unsigned)((n + 255) / 256), 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(
        n, L, jac, g_delta, g_L);
    return check(hipGetLastError());
}
