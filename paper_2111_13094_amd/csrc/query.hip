// query.hip -- conditioning of fitted 5-D mixtures on a position, the solid-angle pdf of
// the conditioned directional mixture, and sampling from it, on gfx950.
//
// Method (Dodik et al., arXiv 2111.13094): joint fit conditioned on the position with the
// standard closed-form Gaussian conditioning (Sec. 3.2 first paragraph, Sec. 3.3); mixture
// pdf with respect to solid angle (Sec. 3.1, with the change of variables dividing the
// tangent density by sinc|nu|); sampling by component, tangent Gaussian and exp map, with
// draws beyond the cut locus |nu| >= pi discarded (Sec. 3.1, "Sampling").
//
// Lane mapping as in the E-step: a wave holds 64/G queries (or draws) x G component lanes;
// normalisations and mixture sums are DPP all-reduces inside the G-lane group.
#include <algorithm>

#include "common.hpp"
#include "query_common.hpp"
#include "timing.hpp"

namespace sdmm {

__global__ void cond_prepare_kernel(int C, int K, const double* __restrict__ pi, const double* __restrict__ mud,
                                    const double* __restrict__ mux, const double* __restrict__ cov,
                                    float* __restrict__ table)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)C * K) return;
    const double* S = cov + 15 * g;
    float T[kCond];
    // chunk q of component k of cell c at ((c * 8 + q) * K + k) * 4 floats
    float4* dst = reinterpret_cast<float4*>(table + (g / K) * K * kCond + (g % K) * 4);
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < kCond / 4; ++q)
            dst[(int64_t)q * K] = make_float4(T[4 * q], T[4 * q + 1], T[4 * q + 2], T[4 * q + 3]);
    };
    bool ok = isfinite(pi[g]) && pi[g] >= 0.0;
    for (int d = 0; d < 3; ++d) ok = ok && isfinite(mud[3 * g + d]) && isfinite(mux[3 * g + d]);
    double Sxx[6], Lxx[6], Lxi[6], Sp[3], Lp[3], Lpi[3];
    for (int d = 0; d < 3; ++d)
        for (int e = 0; e <= d; ++e) Sxx[tri(d, e)] = S[tri(2 + d, 2 + e)];
    ok = ok && chol64<3>(Sxx, Lxx);
    double A[6] = {0, 0, 0, 0, 0, 0};
    if (ok) {
        tri_inv64<3>(Lxx, Lxi);
        // Wm = Lxx^-1 Sigma_xn (3x2); A = Wm^T Lxx^-1; Sigma' = Sigma_nn - Wm^T Wm
        double Wm[3][2];
        for (int d = 0; d < 3; ++d)
            for (int a = 0; a < 2; ++a) {
                double s = 0.0;
                for (int e = 0; e <= d; ++e) s += Lxi[tri(d, e)] * S[tri(2 + e, a)];
                Wm[d][a] = s;
            }
        for (int a = 0; a < 2; ++a)
            for (int d = 0; d < 3; ++d) {
                double s = 0.0;
                for (int e = d; e < 3; ++e) s += Wm[e][a] * Lxi[tri(e, d)];
                A[3 * a + d] = s;
            }
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b <= a; ++b)
                Sp[tri(a, b)] = S[tri(a, b)] - (Wm[0][a] * Wm[0][b] + Wm[1][a] * Wm[1][b] + Wm[2][a] * Wm[2][b]);
        ok = chol64<2>(Sp, Lp);
    }
    double R[9];
    if (ok) {
        frame64(mud + 3 * g, R);
        tri_inv64<2>(Lp, Lpi);
    }
    const double kap = sqrt(0.5 * kLog2e);
    if (!ok) {
        for (int i = 0; i < kCond; ++i) T[i] = 0.0f;
        T[0] = T[4] = T[8] = 1.0f;
        T[12] = T[14] = T[17] = 1.0f;
        T[24] = T[26] = T[27] = T[29] = 1.0f;
        T[30] = -INFINITY;
        store();
        return;
    }
    for (int i = 0; i < 9; ++i) T[i] = (float)R[i];
    for (int d = 0; d < 3; ++d) T[9 + d] = (float)mux[3 * g + d];
    for (int i = 0; i < 6; ++i) T[12 + i] = (float)(Lxi[i] * kap);
    for (int i = 0; i < 6; ++i) T[18 + i] = (float)A[i];
    for (int i = 0; i < 3; ++i) T[24 + i] = (float)Lp[i];
    for (int i = 0; i < 3; ++i) T[27 + i] = (float)(Lpi[i] * kap);
    const double ldx = log(Lxx[0]) + log(Lxx[2]) + log(Lxx[5]);
    T[30] = (float)((log(pi[g]) - ldx - 1.5 * kLn2Pi) * kLog2e);
    T[31] = (float)((-(log(Lp[0]) + log(Lp[2])) - kLn2Pi) * kLog2e);
    store();
}

// pi'_k N2(nu_k - m_k; 0, Sigma'_k) / sinc|nu_k| at direction w (0 at the cut locus), with
// lc = log2 pi'_k + T[31] (pdf_log_const; -inf for a component of weight zero)
__device__ __forceinline__ float pdf_component(const float* T, float lc, float m0, float m1, float wx, float wy,
                                               float wz)
{
    // the 1e-18 offset of the log map rides on the rotation's first row
    const float xr = fmaf(T[0], wx, fmaf(T[1], wy, fmaf(T[2], wz, 1e-18f)));
    const float yr = fmaf(T[3], wx, fmaf(T[4], wy, T[5] * wz));
    const float zr = fmaf(T[6], wx, fmaf(T[7], wy, T[8] * wz));
    float n0, n1;
    const float f = log_map_f32_offset(xr, yr, zr, n0, n1);
    const float r2 = fmaf(n0, n0, n1 * n1);
    const float d0 = n0 - m0, d1 = n1 - m1;
    const float u0 = T[27] * d0;
    const float u1 = fmaf(T[28], d0, T[29] * d1);
    const float q = fmaf(u0, u0, u1 * u1);
    const float p = __builtin_amdgcn_exp2f(lc - q) * f;
    return r2 < kCutSq ? p : 0.0f;
}

// log2 of the conditioned weight plus the conditional density's log2 normaliser T[31]
__device__ __forceinline__ float pdf_log_const(const float* T, float wk)
{
    return T[31] + __builtin_amdgcn_logf(wk);
}

// One draw for the group's query: pick the component by the CDF of pi' (prefix sum in
// component order, lowest index on ties), sample nu = m + L' z (Box-Muller), discard at
// |nu| >= pi, map with the exp map, evaluate the conditioned pdf at the result.
template <int G>
__device__ __forceinline__ void sample_one(const float* T, bool usable, float wk, float m0, float m1, int K,
                                           float u0, float u1, float u2, float& ox, float& oy, float& oz,
                                           float& pdf, int& valid, int& comp_sel)
{
    const int lane = threadIdx.x & 63;
    const int comp = lane % G, base = lane - comp;
    const float cdf = group_inclusive_scan<G>(wk);
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << base);
    const uint64_t hit = __ballot(comp < K && usable && u0 < cdf) & gmask;
    const uint64_t pos = __ballot(comp < K && usable && wk > 0.0f) & gmask;
    int sel = -1;
    if (hit) sel = __builtin_ctzll(hit) - base;
    else if (pos) sel = 63 - __builtin_clzll(pos) - base;
    // every lane forms its own component's candidate; the selected one is broadcast
    float w[3];
    const int ok = draw_candidate(T, T[24], T[25], T[26], m0, m1, u1, u2, w);
    const int src = base + (sel < 0 ? 0 : sel);
    ox = __shfl(w[0], src);
    oy = __shfl(w[1], src);
    oz = __shfl(w[2], src);
    valid = (sel >= 0) ? __shfl(ok, src) : 0;
    comp_sel = sel;
    const float c = pdf_component(T, pdf_log_const(T, wk), m0, m1, ox, oy, oz);
    pdf = group_sum<G>(comp < K ? c : 0.0f);
    if (!valid) {
        ox = oy = oz = 0.0f;
        pdf = 0.0f;
    }
}

// ---------------------------------------------------------------------------------
// kernels: the loop trip count is uniform per wave so every group reaches the DPP steps
// ---------------------------------------------------------------------------------
template <int G>
__global__ __launch_bounds__(256) void condition_kernel(const float* __restrict__ table, int C, int K,
                                                        const float* __restrict__ qpos, const int32_t* __restrict__ qcell,
                                                        int64_t nq, float* __restrict__ cw, float* __restrict__ cm)
{
    constexpr int S = 64 / G;
    const int lane = threadIdx.x & 63, comp = lane % G, slot = lane / G;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t q0 = wave * S; q0 < nq; q0 += nwaves * S) {
        const int64_t q = q0 + slot;
        const bool inq = q < nq;
        const int qc = inq ? qcell[q] : 0;
        const bool usable = inq && qc >= 0 && qc < C;
        float T[kCond];
        load_row(table_row(table, qc, K, comp, usable), K, T);
        const int64_t qq = inq ? q : 0;
        float m0, m1;
        float lw = cond_component(T, qpos[qq], qpos[nq + qq], qpos[2 * nq + qq], m0, m1);
        if (comp >= K || !usable) lw = -INFINITY;
        const float wk = cond_weight<G>(lw);
        if (inq && comp < K) {
            cw[q * K + comp] = wk;
            cm[(q * K + comp) * 2] = usable ? m0 : 0.0f;
            cm[(q * K + comp) * 2 + 1] = usable ? m1 : 0.0f;
        }
    }
}

template <int G>
__global__ __launch_bounds__(256) void pdf_kernel(const float* __restrict__ table, int C, int K,
                                                  const int32_t* __restrict__ qcell, int64_t nq,
                                                  const float* __restrict__ cw, const float* __restrict__ cm, int nd,
                                                  const float* __restrict__ dirs, float* __restrict__ pdf_out)
{
    constexpr int S = 64 / G;
    const int lane = threadIdx.x & 63, comp = lane % G, slot = lane / G;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t np = nq * nd;
    for (int64_t p0 = wave * S; p0 < np; p0 += nwaves * S) {
        const int64_t p = p0 + slot;
        const bool inp = p < np;
        const int64_t pp = inp ? p : 0;
        const int64_t q = pp / nd;
        const int qc = qcell[q];
        const bool usable = inp && qc >= 0 && qc < C && comp < K;
        float T[kCond];
        load_row(table_row(table, qc, K, comp, usable), K, T);
        const int kk = comp < K ? comp : K - 1;
        const float wk = usable ? cw[q * K + kk] : 0.0f;
        const float m0 = cm[(q * K + kk) * 2], m1 = cm[(q * K + kk) * 2 + 1];
        const float c = pdf_component(T, pdf_log_const(T, wk), m0, m1, dirs[pp], dirs[np + pp], dirs[2 * np + pp]);
        const float tot = group_sum<G>(usable ? c : 0.0f);
        if (inp && comp == 0) pdf_out[p] = tot;
    }
}

template <int G>
__global__ __launch_bounds__(256) void sample_kernel(const float* __restrict__ table, int C, int K,
                                                     const int32_t* __restrict__ qcell, int64_t nq,
                                                     const float* __restrict__ cw, const float* __restrict__ cm,
                                                     int ns, const float* __restrict__ uniforms, uint64_t seed,
                                                     float* __restrict__ dirs_out, float* __restrict__ pdf_out,
                                                     uint8_t* __restrict__ valid_out, int32_t* __restrict__ comp_out)
{
    constexpr int S = 64 / G;
    const int lane = threadIdx.x & 63, comp = lane % G, slot = lane / G;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t nd = nq * ns;
    for (int64_t d0 = wave * S; d0 < nd; d0 += nwaves * S) {
        const int64_t d = d0 + slot;
        const bool ind = d < nd;
        const int64_t dd = ind ? d : 0;
        const int64_t q = dd / ns;
        const int qc = qcell[q];
        const bool usable = ind && qc >= 0 && qc < C;
        float T[kCond];
        load_row(table_row(table, qc, K, comp, usable), K, T);
        const int kk = comp < K ? comp : K - 1;
        const float wk = (usable && comp < K) ? cw[q * K + kk] : 0.0f;
        const float m0 = cm[(q * K + kk) * 2], m1 = cm[(q * K + kk) * 2 + 1];
        float u0, u1, u2;
        draw_uniforms(uniforms, nd, dd, seed, u0, u1, u2);
        float ox, oy, oz, pdf;
        int valid, sel;
        sample_one<G>(T, usable, wk, m0, m1, K, u0, u1, u2, ox, oy, oz, pdf, valid, sel);
        if (ind && comp == 0) {
            dirs_out[d] = ox;
            dirs_out[nd + d] = oy;
            dirs_out[2 * nd + d] = oz;
            pdf_out[d] = pdf;
            valid_out[d] = (uint8_t)valid;
            if (comp_out) comp_out[d] = sel;
        }
    }
}

// conditioning + ns draws + pdf per query, pi' and m kept in registers. The draws of a
// query are taken G at a time, draw t0 + c by lane c of the query's group: the group
// picks every draw's component against the query's CDF (one scan per query), lane c
// gathers its draw's component row (frame, conditional factor and mean) from the lane
// that holds it and forms the candidate, and the group then evaluates the pdf of each
// draw's direction over all components. The arithmetic of every value is the one of
// sample_one, so both paths give the same draws.
template <int G>
__global__ __launch_bounds__(256) void cond_sample_pdf_kernel(const float* __restrict__ table, int C, int K,
                                                              const float* __restrict__ qpos,
                                                              const int32_t* __restrict__ qcell, int64_t nq, int ns,
                                                              const float* __restrict__ uniforms, uint64_t seed,
                                                              float* __restrict__ dirs_out, float* __restrict__ pdf_out,
                                                              uint8_t* __restrict__ valid_out)
{
    constexpr int S = 64 / G;
    const int lane = threadIdx.x & 63, comp = lane % G, slot = lane / G, base = lane - comp;
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << base);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t nd = nq * ns;
    for (int64_t q0 = wave * S; q0 < nq; q0 += nwaves * S) {
        const int64_t q = q0 + slot;
        const bool inq = q < nq;
        const int64_t qq = inq ? q : 0;
        const int qc = qcell[qq];
        const bool usable = inq && qc >= 0 && qc < C;
        float T[kCond];
        load_row(table_row(table, qc, K, comp, usable), K, T);
        float m0, m1;
        float lw = cond_component(T, qpos[qq], qpos[nq + qq], qpos[2 * nq + qq], m0, m1);
        if (comp >= K || !usable) lw = -INFINITY;
        const float wk = cond_weight<G>(lw);
        const float lc = pdf_log_const(T, wk);
        const float cdf = group_inclusive_scan<G>(wk);
        const bool cand = comp < K && usable;
        const uint64_t pos = __ballot(cand && wk > 0.0f) & gmask;
        const int last_pos = pos ? 63 - __builtin_clzll(pos) - base : -1;
        for (int t0 = 0; t0 < ns; t0 += G) {
            float ul0 = 0.0f, ul1 = 0.0f, ul2 = 0.0f;
            if (t0 + comp < ns) draw_uniforms(uniforms, nd, qq * ns + t0 + comp, seed, ul0, ul1, ul2);
            const int tn = min(G, ns - t0);  // wave-uniform
            // four draws at a time, so that their independent chains interleave (a draw
            // past tn repeats the last one and is not kept)
            int sel = -1;
            for (int tt = 0; tt < tn; tt += 4) {
                float u0[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) u0[j] = __shfl(ul0, base + min(tt + j, tn - 1));
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint64_t hit = __ballot(cand && u0[j] < cdf) & gmask;
                    const int s_tt = hit ? __builtin_ctzll(hit) - base : last_pos;
                    sel = comp == tt + j ? s_tt : sel;
                }
            }
            const int src = base + (sel < 0 ? 0 : sel);
            float R[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) R[i] = __shfl(T[i], src);
            const float l0 = __shfl(T[24], src), l1 = __shfl(T[25], src), l2 = __shfl(T[26], src);
            float w[3];
            const int ok = draw_candidate(R, l0, l1, l2, __shfl(m0, src), __shfl(m1, src), ul1, ul2, w);
            const int valid = sel >= 0 && ok;
            float pdf = 0.0f;
            for (int tt = 0; tt < tn; tt += 4) {
                float c[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int from = base + min(tt + j, tn - 1);
                    c[j] = pdf_component(T, lc, m0, m1, __shfl(w[0], from), __shfl(w[1], from), __shfl(w[2], from));
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float p = group_sum<G>(comp < K ? c[j] : 0.0f);
                    pdf = comp == tt + j ? p : pdf;
                }
            }
            if (inq && comp < tn) {
                const int64_t d = qq * ns + t0 + comp;
                dirs_out[d] = valid ? w[0] : 0.0f;
                dirs_out[nd + d] = valid ? w[1] : 0.0f;
                dirs_out[2 * nd + d] = valid ? w[2] : 0.0f;
                pdf_out[d] = valid ? pdf : 0.0f;
                valid_out[d] = (uint8_t)valid;
            }
        }
    }
}

// The same conditioning, draws and pdf as cond_sample_pdf_kernel, in three wave-local
// phases over QB = S * NQR queries, NQR rounds of S queries with QB * ns <= 64 draws:
//   A. conditioning, lane = (query slot, component), per round: pi', the CDF of pi' and
//      m into LDS, with each query's cell and last component of positive weight;
//   B. the draws, one per lane: uniforms, the component by the CDF, the candidate from
//      the table row of that component;
//   C. the pdf, lane = (query slot, component) again: every draw of the query over all
//      components, four at a time.
// Phase B runs on every lane instead of on ns of each query's G lanes. The draws are
// computed by the same arithmetic as in sample_one (the scan, the first CDF entry above
// u0, draw_candidate), so they are the same; the pdf sums over the components may
// associate differently (FP32 rounding).
template <int G>
__global__ __launch_bounds__(256) void cond_sample_pdf_lanes_kernel(const float* __restrict__ table, int C, int K,
                                                                    const float* __restrict__ qpos,
                                                                    const int32_t* __restrict__ qcell, int64_t nq,
                                                                    int ns, int nqr, const float* __restrict__ uniforms,
                                                                    uint64_t seed, float* __restrict__ dirs_out,
                                                                    float* __restrict__ pdf_out,
                                                                    uint8_t* __restrict__ valid_out)
{
    constexpr int S = 64 / G, QBMAX = 4 * S, WPB = 4;
    // per wave: the CDF of pi' (-inf past K and for unusable queries, so that no draw
    // picks those lanes), the pdf's log constants and the conditioned means of its
    // queries' components; each query's cell (-1: none) and last component of positive
    // weight; the draws' directions and validity
    __shared__ __align__(16) float cdf_s[WPB][QBMAX][G];
    __shared__ float lc_s[WPB][QBMAX][G], m0_s[WPB][QBMAX][G], m1_s[WPB][QBMAX][G];
    __shared__ int last_s[WPB][QBMAX], cell_s[WPB][QBMAX];
    __shared__ float4 w_s[WPB][64];
    __shared__ int valid_s[WPB][64];
    const int lane = threadIdx.x & 63, comp = lane % G, slot = lane / G, base = lane - comp;
    const int wv = threadIdx.x >> 6;
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << base);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t nd = nq * ns;
    const int QB = S * nqr;
    // the lane's table row stays in registers while its queries' cell repeats (queries
    // sorted by cell mostly share one); `row_cell` is the cell it holds
    float T[kCond];
    int row_cell = -1;
    auto row_for = [&](int cell) {
        if (cell != row_cell) {
            load_row(table_row(table, cell, K, comp, true), K, T);
            row_cell = cell;
        }
    };
    for (int64_t qb = wave * QB; qb < nq; qb += nwaves * QB) {
        // A: conditioning
        for (int r = 0; r < nqr; ++r) {
            const int qi = r * S + slot;
            const int64_t q = qb + qi;
            const bool inq = q < nq;
            const int64_t qq = inq ? q : 0;
            const int qc = qcell[qq];
            const bool usable = inq && qc >= 0 && qc < C;
            row_for(usable ? qc : 0);
            float m0, m1;
            float lw = cond_component(T, qpos[qq], qpos[nq + qq], qpos[2 * nq + qq], m0, m1);
            if (comp >= K || !usable) lw = -INFINITY;
            const float wk = cond_weight<G>(lw);
            const float cdf = group_inclusive_scan<G>(wk);
            const uint64_t pos = __ballot(comp < K && usable && wk > 0.0f) & gmask;
            cdf_s[wv][qi][comp] = (comp < K && usable) ? cdf : -INFINITY;
            lc_s[wv][qi][comp] = pdf_log_const(T, wk);
            m0_s[wv][qi][comp] = m0;
            m1_s[wv][qi][comp] = m1;
            if (comp == 0) {
                last_s[wv][qi] = pos ? 63 - __builtin_clzll(pos) - base : -1;
                cell_s[wv][qi] = usable ? qc : -1;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // this wave's LDS writes are done
        // B: one draw per lane
        {
            const int qi = lane / ns, t = lane % ns;
            const int64_t q = qb + qi;
            const bool act = qi < QB && q < nq;
            const int64_t d = act ? q * ns + t : 0;
            float u0, u1, u2;
            draw_uniforms(uniforms, nd, d, seed, u0, u1, u2);
            const int qis = act ? qi : 0;
            const int qc = cell_s[wv][qis];
            // the first component whose CDF value exceeds u0, else the last of positive weight
            int first = -1;
            const float4* crow = reinterpret_cast<const float4*>(&cdf_s[wv][qis][0]);
#pragma unroll
            for (int c4 = G / 4 - 1; c4 >= 0; --c4) {
                const float4 v = crow[c4];
                first = u0 < v.w ? 4 * c4 + 3 : first;
                first = u0 < v.z ? 4 * c4 + 2 : first;
                first = u0 < v.y ? 4 * c4 + 1 : first;
                first = u0 < v.x ? 4 * c4 : first;
            }
            const int sel = first >= 0 ? first : last_s[wv][qis];
            const int sk = sel < 0 ? 0 : sel;
            const float4* row = reinterpret_cast<const float4*>(table_row(table, qc, K, sk, qc >= 0));
            float R[12];
#pragma unroll
            for (int c4 = 0; c4 < 3; ++c4) {
                const float4 v = row[(int64_t)c4 * K];
                R[4 * c4] = v.x;
                R[4 * c4 + 1] = v.y;
                R[4 * c4 + 2] = v.z;
                R[4 * c4 + 3] = v.w;
            }
            const float4 lp = row[(int64_t)6 * K];  // T24-T27: L' packed and one more
            float w[3];
            const int ok = draw_candidate(R, lp.x, lp.y, lp.z, m0_s[wv][qis][sk], m1_s[wv][qis][sk], u1, u2, w);
            const int valid = act && sel >= 0 && ok;
            w_s[wv][lane] = make_float4(w[0], w[1], w[2], 0.0f);
            valid_s[wv][lane] = valid;
            if (act) {  // the pass's draws are contiguous: d = qb * ns + lane
                dirs_out[d] = valid ? w[0] : 0.0f;
                dirs_out[nd + d] = valid ? w[1] : 0.0f;
                dirs_out[2 * nd + d] = valid ? w[2] : 0.0f;
                valid_out[d] = (uint8_t)valid;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        // C: the pdf of every draw over all components, outputs
        for (int r = 0; r < nqr; ++r) {
            const int qi = r * S + slot;
            const int64_t q = qb + qi;
            const bool inq = q < nq;
            const int qc = cell_s[wv][qi];
            row_for(qc >= 0 ? qc : 0);
            const float lc = lc_s[wv][qi][comp], m0 = m0_s[wv][qi][comp], m1 = m1_s[wv][qi][comp];
            float pdf = 0.0f;
            for (int tt = 0; tt < ns; tt += 4) {  // wave-uniform
                float c[4];
                const float4* wq = &w_s[wv][qi * ns + tt];
                if (tt + 4 <= ns) {  // four draws of this query
#pragma unroll
                    for (int j = 0; j < 4; ++j) c[j] = pdf_component(T, lc, m0, m1, wq[j].x, wq[j].y, wq[j].z);
                } else {  // the last ones, repeated up to four
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float4 wd = wq[min(j, ns - 1 - tt)];
                        c[j] = pdf_component(T, lc, m0, m1, wd.x, wd.y, wd.z);
                    }
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) c[j] = comp < K ? c[j] : 0.0f;
                if constexpr (G == 16) {
                    // the four sums over the row at once: lane comp ends with the sum for
                    // draw tt + (comp & 3) (group_sum4_row16), kept by the quad of that draw
                    const float p = group_sum4_row16(c);
                    pdf = (comp >> 2) == (tt >> 2) ? p : pdf;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float p = group_sum<G>(c[j]);
                        pdf = comp == tt + j ? p : pdf;
                    }
                }
            }
            if (inq && comp < ns) pdf_out[q * ns + comp] = valid_s[wv][qi * ns + comp] ? pdf : 0.0f;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // before the next pass overwrites
    }
}

}  // namespace sdmm

using namespace sdmm;

extern "C" int sdmm_condition_prepare(const sdmm_mixtures* mix, float* table, void* stream)
{
    if (!mix || !table || mix->n_cells <= 0 || mix->K < 1 || mix->K > kMaxK) return SDMM_EINVAL;
    if (!mix->weights || !mix->mean_dir || !mix->mean_pos || !mix->cov) return SDMM_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t nk = (int64_t)mix->n_cells * mix->K;
    cond_prepare_kernel<<<(unsigned)((nk + 255) / 256), 256, 0, s>>>(mix->n_cells, mix->K, mix->weights,
                                                                      mix->mean_dir, mix->mean_pos, mix->cov, table);
    return check(hipGetLastError());
}

extern "C" int sdmm_condition(const float* table, int32_t n_cells, int32_t K, const float* qpos,
                              const int32_t* qcell, int64_t nq, float* cond_w, float* cond_m, void* stream)
{
    if (!table || n_cells <= 0 || K < 1 || K > kMaxK || nq < 0) return SDMM_EINVAL;
    if (nq == 0) return SDMM_OK;
    if (!qpos || !qcell || !cond_w || !cond_m) return SDMM_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int G = group_for(K);
    SDMM_DISPATCH_G(G, (condition_kernel<g><<<grid_for(nq, 64 / g), 256, 0, s>>>(table, n_cells, K, qpos, qcell,
                                                                                  nq, cond_w, cond_m)));
    return check(hipGetLastError());
}

extern "C" int sdmm_pdf(const float* table, int32_t n_cells, int32_t K, const int32_t* qcell, int64_t nq,
                        const float* cond_w, const float* cond_m, int32_t nd, const float* dirs, float* pdf_out,
                        void* stream)
{
    if (!table || n_cells <= 0 || K < 1 || K > kMaxK || nq < 0 || nd < 0) return SDMM_EINVAL;
    if (nq == 0 || nd == 0) return SDMM_OK;
    if (!qcell || !cond_w || !cond_m || !dirs || !pdf_out) return SDMM_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int G = group_for(K);
    SDMM_DISPATCH_G(G, (pdf_kernel<g><<<grid_for(nq * nd, 64 / g), 256, 0, s>>>(table, n_cells, K, qcell, nq, cond_w,
                                                                                 cond_m, nd, dirs, pdf_out)));
    return check(hipGetLastError());
}

extern "C" int sdmm_sample(const float* table, int32_t n_cells, int32_t K, const int32_t* qcell, int64_t nq,
                           const float* cond_w, const float* cond_m, int32_t ns, const float* uniforms,
                           uint64_t seed, float* dirs_out, float* pdf_out, uint8_t* valid_out, int32_t* comp_out,
                           void* stream)
{
    if (!table || n_cells <= 0 || K < 1 || K > kMaxK || nq < 0 || ns < 0) return SDMM_EINVAL;
    if (nq == 0 || ns == 0) return SDMM_OK;
    if (!qcell || !cond_w || !cond_m || !dirs_out || !pdf_out || !valid_out) return SDMM_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int G = group_for(K);
    SDMM_DISPATCH_G(G, (sample_kernel<g><<<grid_for(nq * ns, 64 / g), 256, 0, s>>>(
                           table, n_cells, K, qcell, nq, cond_w, cond_m, ns, uniforms, seed, dirs_out, pdf_out,
                           valid_out, comp_out)));
    return check(hipGetLastError());
}

extern "C" int sdmm_condition_sample_pdf(const float* table, int32_t n_cells, int32_t K, const float* qpos,
                                         const int32_t* qcell, int64_t nq, int32_t ns, const float* uniforms,
                                         uint64_t seed, float* dirs_out, float* pdf_out, uint8_t* valid_out,
                                         void* stream)
{
    if (!table || n_cells <= 0 || K < 1 || K > kMaxK || nq < 0 || ns < 0) return SDMM_EINVAL;
    if (nq == 0 || ns == 0) return SDMM_OK;
    if (!qpos || !qcell || !dirs_out || !pdf_out || !valid_out) return SDMM_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int G = group_for(K);
    ScopedTimer tm(SDMM_TIMER_QUERY, s);
    const int S = 64 / G;
    if (S * ns <= 64) {
        // draws of up to four rounds of S queries share one pass of the draw phase
        const int nqr = std::max(1, std::min(4, 64 / (S * ns)));
        SDMM_DISPATCH_G(G, (cond_sample_pdf_lanes_kernel<g><<<grid_for(nq, S * nqr), 256, 0, s>>>(
                               table, n_cells, K, qpos, qcell, nq, ns, nqr, uniforms, seed, dirs_out, pdf_out,
                               valid_out)));
    } else {
        SDMM_DISPATCH_G(G, (cond_sample_pdf_kernel<g><<<grid_for(nq, 64 / g), 256, 0, s>>>(
                               table, n_cells, K, qpos, qcell, nq, ns, uniforms, seed, dirs_out, pdf_out, valid_out)));
    }
    return check(hipGetLastError());
}
