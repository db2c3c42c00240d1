// estep.hpp -- the E-step pass over one work item (a chunk of one cell's samples), shared
// by the EM kernels and the adjoint kernel.
//
// For every (sample i, component k) pair of the chunk (Sec. 3.1, 3.2 of Dodik et al.):
//   y_ik = (log_{mu_k}(w_i), p_i - mu_x_k),
//   l_ik = log2 pi_k N5(y_ik; 0, Sigma_k) through the scaled inverse Cholesky factor,
//   r_ik = exp2(l_ik - max_k l) / sum_k exp2(l_ik - max_k l)   (DPP all-reduce in the group),
//   S0 += w r, S1 += w r y, S2 += w r y y^T (packed).
// With ADJ it also accumulates sum_i w_i log p(y_i) and the directional-mean gradient
// terms sum w r (d nu / d delta)^T (L^-T z)_nu for the adjoint.
#pragma once

#include "device_math.hpp"

namespace sdmm {

enum { kAccTwoSum = 0, kAccPlain = 1, kAccFp64 = 2 };
constexpr int kFoldEvery = 32;  // steps between folds of the FP32 block sums

// running sums: FP32 block sums over kFoldEvery steps, folded into an FP32 TwoSum pair
// (compensated), kept as one plain FP32 sum, or folded into FP64 (precision variants)
template <int ACC>
struct RunSum;

template <>
struct RunSum<kAccTwoSum> {
    float blk = 0.0f, hi = 0.0f, lo = 0.0f;
    __device__ __forceinline__ void add(float v) { blk += v; }
    __device__ __forceinline__ void fma_add(float a, float b) { blk = fmaf(a, b, blk); }
    __device__ __forceinline__ void fold()
    {
        const float s = hi + blk;
        const float bb = s - hi;
        const float err = (hi - (s - bb)) + (blk - bb);
        hi = s;
        lo += err;
        blk = 0.0f;
    }
    __device__ __forceinline__ double total()
    {
        fold();
        return (double)hi + (double)lo;
    }
};

template <>
struct RunSum<kAccPlain> {
    float blk = 0.0f;
    __device__ __forceinline__ void add(float v) { blk += v; }
    __device__ __forceinline__ void fma_add(float a, float b) { blk = fmaf(a, b, blk); }
    __device__ __forceinline__ void fold() {}
    __device__ __forceinline__ double total() { return (double)blk; }
};

template <>
struct RunSum<kAccFp64> {
    float blk = 0.0f;
    double hi = 0.0;
    __device__ __forceinline__ void add(float v) { blk += v; }
    __device__ __forceinline__ void fma_add(float a, float b) { blk = fmaf(a, b, blk); }
    __device__ __forceinline__ void fold()
    {
        hi += (double)blk;
        blk = 0.0f;
    }
    __device__ __forceinline__ double total()
    {
        fold();
        return hi;
    }
};

// statistics per component and the per-chunk record layout
template <bool ADJ>
struct ChunkLayout {
    static constexpr int kNStat = ADJ ? 23 : 21;       // S0, S1[5], S2[15] (+ g_delta[2])
    static constexpr int kNRed = kNStat + (ADJ ? 4 : 3); // + W, M, negatives (+ LL)
    static __host__ __device__ constexpr int record(int K) { return (kNStat * K + (kNRed - kNStat) + 1) & ~1; }
};

// Twist of the frame about mu when mu moves along its own tangent directions:
// phi_j = (d t1 / d mu . t_j) . t2 for the basis of frame64 (Duff et al. 2017), so that
// moving mu by delta_j t_j turns (t1, t2) by phi_j about mu, besides tilting it.
__device__ __forceinline__ void frame_twist64(const double mu[3], const double R[9], double phi[2])
{
    const double sg = copysign(1.0, mu[2]);
    const double a = -1.0 / (sg + mu[2]);
    const double a2 = a * a;
    const double nx = mu[0], ny = mu[1];
    const double db[3] = {ny * a, nx * a, nx * ny * a2};
    const double dt1[9] = {2.0 * sg * nx * a, 0.0, sg * nx * nx * a2, sg * db[0], sg * db[1], sg * db[2],
                           -sg, 0.0, 0.0};
    for (int j = 0; j < 2; ++j) {
        const double* tj = R + 3 * j;
        double v[3];
        for (int r = 0; r < 3; ++r) v[r] = dt1[3 * r] * tj[0] + dt1[3 * r + 1] * tj[1] + dt1[3 * r + 2] * tj[2];
        phi[j] = v[0] * R[3] + v[1] * R[4] + v[2] * R[5];
    }
}

// ---------------------------------------------------------------------------------
// FP32 E-step mirror of one component: R (9), mu_x (3), Linv * sqrt(log2(e)/2) (15),
// c * log2(e) with c = log pi - log det L - (5/2) log 2 pi (1), the frame twist rates (2)
// used by the adjoint, and the FP32 rounding residues of R (9) and mu_x (3), with which
// the adjoint pass forms tangent coordinates to FP32 relative accuracy (its gradients
// are small differences near stationarity). Returns false and writes an inert mirror
// (identity frame and factor) when the component is unusable.
// ---------------------------------------------------------------------------------
__device__ inline bool write_mirror(double pi, const double* mud, const double* mux, const double* cov,
                             float* out)
{
    bool ok = isfinite(pi) && pi >= 0.0;
    for (int d = 0; d < 3; ++d) ok = ok && isfinite(mud[d]) && isfinite(mux[d]);
    double L[15], Li[15];
    ok = ok && chol64<5>(cov, L);
    if (!ok) {
        for (int i = 0; i < kMirror; ++i) out[i] = 0.0f;
        out[0] = out[4] = out[8] = 1.0f;
        const int diag[5] = {0, 2, 5, 9, 14};
        for (int d = 0; d < 5; ++d) out[12 + diag[d]] = 1.0f;
        return false;
    }
    double R[9];
    frame64(mud, R);
    tri_inv64<5>(L, Li);
    double logdet = 0.0;
    for (int d = 0; d < 5; ++d) logdet += log(L[tri(d, d)]);
    const double scale = sqrt(0.5 * kLog2e);
    for (int i = 0; i < 9; ++i) out[i] = (float)R[i];
    for (int d = 0; d < 3; ++d) out[9 + d] = (float)mux[d];
    for (int i = 0; i < 15; ++i) out[12 + i] = (float)(Li[i] * scale);
    out[27] = (float)((log(pi) - logdet - 2.5 * kLn2Pi) * kLog2e);
    double phi[2];
    frame_twist64(mud, R, phi);
    out[28] = (float)phi[0];
    out[29] = (float)phi[1];
    out[30] = out[31] = 0.0f;
    for (int i = 0; i < 9; ++i) out[32 + i] = (float)(R[i] - (double)out[i]);
    for (int d = 0; d < 3; ++d) out[41 + d] = (float)(mux[d] - (double)out[9 + d]);
    for (int i = 44; i < kMirror; ++i) out[i] = 0.0f;
    return true;
}

struct SampleRegs {
    float ox, oy, oz, px, py, pz, w;
};

// loads sample ii of a chunk; the seven channel bases are wave-uniform (SGPRs) and the
// lane offset is a 32-bit byte offset, so each load is one saddr+voffset instruction
__device__ __forceinline__ float ld_off(const float* base, uint32_t byte_off)
{
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + byte_off);
}

__device__ __forceinline__ SampleRegs load_sample(const float* const* ch, uint32_t ii)
{
    const uint32_t b = ii * 4u;
    SampleRegs r;
    r.ox = ld_off(ch[0], b);
    r.oy = ld_off(ch[1], b);
    r.oz = ld_off(ch[2], b);
    r.px = ld_off(ch[3], b);
    r.py = ld_off(ch[4], b);
    r.pz = ld_off(ch[5], b);
    r.w = ld_off(ch[6], b);
    return r;
}

// W = sum w (FP64 per lane), M = #{w > 0}, negatives = #{w < 0} over [s0, s1), one
// sample per lane; every lane of the wave returns the wave's totals.
__device__ __forceinline__ void weight_pass(const float* __restrict__ wch, int64_t s0, int64_t s1, double& W,
                                            double& M, double& neg)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    double sw = 0.0;
    int cnt = 0, ng = 0;
    for (int64_t i = s0 + (int64_t)wave * 64 + lane; i < s1; i += (int64_t)nwaves * 64) {
        const float w = wch[i];
        sw += (double)w;
        cnt += w > 0.0f;
        ng += w < 0.0f;
    }
    double c = (double)cnt, g = (double)ng;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        sw += __shfl_xor(sw, o);
        c += __shfl_xor(c, o);
        g += __shfl_xor(g, o);
    }
    W = sw;
    M = c;
    neg = g;
}

// derivative of theta/sin(theta) with respect to z = cos(theta) on the sphere
__device__ __forceinline__ float dtheta_over_sin_dz(float z, float rs)
{
    const float az = fabsf(z);
    // derivative of theta_over_sin_pos (degree-9 polynomial)
    float p = 9.0f * -1.048102602e-02f;
    p = fmaf(p, az, 8.0f * 6.458827853e-02f);
    p = fmaf(p, az, 7.0f * -1.854392439e-01f);
    p = fmaf(p, az, 6.0f * 3.409982324e-01f);
    p = fmaf(p, az, 5.0f * -4.757513404e-01f);
    p = fmaf(p, az, 4.0f * 5.744850039e-01f);
    p = fmaf(p, az, 3.0f * -6.644107103e-01f);
    p = fmaf(p, az, 2.0f * 7.852075100e-01f);
    p = fmaf(p, az, -9.999929667e-01f);
    // z < 0: f = pi / s - g(|z|)  ->  f' = pi z / s^3 + g'(|z|)
    return z < 0.0f ? fmaf(kPiF * z, rs * rs * rs, p) : p;
}

// E-step of one chunk [s0, s1) of a cell. mirror_cell points at the cell's K FP32
// mirrors. Writes the chunk record part[] (FP64). lds: nwaves * kNRed * G doubles.
template <int G, int ACC, bool JAC, bool ADJ>
__device__ __forceinline__ void estep_chunk(const float* __restrict__ smp, int64_t N, int64_t s0,
                                            int64_t s1, const float* __restrict__ mirror_cell, int K,
                                            double* __restrict__ part, double* lds)
{
    using CL = ChunkLayout<ADJ>;
    constexpr int NS = CL::kNStat, NR = CL::kNRed;
    constexpr int S = 64 / G;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int comp = lane % G, slot = lane / G;
    const int kk = comp < K ? comp : K - 1;

    const float4* mp = reinterpret_cast<const float4*>(mirror_cell + (int64_t)kk * kMirror);
    float P[44];
#pragma unroll
    for (int q = 0; q < (ADJ ? 11 : 7); ++q) {
        const float4 v = mp[q];
        P[4 * q] = v.x;
        P[4 * q + 1] = v.y;
        P[4 * q + 2] = v.z;
        P[4 * q + 3] = v.w;
    }
    const float c2 = comp < K ? P[27] : -INFINITY;

    // channel bases start at the chunk so that lane offsets fit in 32 bits
    const float* ch[7];
#pragma unroll
    for (int a = 0; a < 7; ++a) ch[a] = smp + (int64_t)a * N + s0;

    RunSum<ACC> acc[NS];
    RunSum<ACC> accll;

    const int64_t n = s1 - s0;
    const int64_t stride = (int64_t)nwaves * S;
    const int64_t steps = (n + stride - 1) / stride;
    const uint32_t last = (uint32_t)(n > 0 ? n - 1 : 0);
    const uint32_t ustride = (uint32_t)stride;

    // one (sample, component) pair per lane
    auto body = [&](const SampleRegs& cur, bool valid) {
        const float w = valid ? cur.w : 0.0f;

        // tangent coordinates y = (log_mu w, p - mu_x)
        float xr = fmaf(P[0], cur.ox, fmaf(P[1], cur.oy, P[2] * cur.oz));
        float yr = fmaf(P[3], cur.ox, fmaf(P[4], cur.oy, P[5] * cur.oz));
        float zr = fmaf(P[6], cur.ox, fmaf(P[7], cur.oy, P[8] * cur.oz));
        if constexpr (ADJ) {  // add the residue of the FP32-rounded frame
            xr += fmaf(P[32], cur.ox, fmaf(P[33], cur.oy, P[34] * cur.oz));
            yr += fmaf(P[35], cur.ox, fmaf(P[36], cur.oy, P[37] * cur.oz));
            zr += fmaf(P[38], cur.ox, fmaf(P[39], cur.oy, P[40] * cur.oz));
        }
        float y0, y1;
        const float f = log_map_f32(xr, yr, zr, y0, y1);
        float y2 = cur.px - P[9], y3 = cur.py - P[10], y4 = cur.pz - P[11];
        if constexpr (ADJ) {
            y2 -= P[41];
            y3 -= P[42];
            y4 -= P[43];
        }

        // log2 of pi_k N5(y; 0, Sigma_k) through the scaled inverse Cholesky factor
        const float z0 = P[12] * y0;
        const float z1 = fmaf(P[13], y0, P[14] * y1);
        const float z2 = fmaf(P[15], y0, fmaf(P[16], y1, P[17] * y2));
        const float z3 = fmaf(P[18], y0, fmaf(P[19], y1, fmaf(P[20], y2, P[21] * y3)));
        const float z4 = fmaf(P[22], y0, fmaf(P[23], y1, fmaf(P[24], y2, fmaf(P[25], y3, P[26] * y4))));
        float l = fmaf(-z0, z0, c2);
        l = fmaf(-z1, z1, l);
        l = fmaf(-z2, z2, l);
        l = fmaf(-z3, z3, l);
        l = fmaf(-z4, z4, l);
        if constexpr (JAC) l += __log2f(f);  // solid-angle density: divide by sinc|nu| = times f

        // responsibilities: log-sum-exp across the component lanes of this sample
        const float lmax = group_max<G>(l);
        const float e = __builtin_amdgcn_exp2f(l - lmax);
        const float den = group_sum<G>(e);
        const float wr = w * (e * __builtin_amdgcn_rcpf(den));

        const float t0 = wr * y0, t1 = wr * y1, t2 = wr * y2, t3 = wr * y3, t4 = wr * y4;
        acc[0].add(wr);
        acc[1].add(t0);
        acc[2].add(t1);
        acc[3].add(t2);
        acc[4].add(t3);
        acc[5].add(t4);
        acc[6].fma_add(t0, y0);
        acc[7].fma_add(t1, y0);
        acc[8].fma_add(t1, y1);
        acc[9].fma_add(t2, y0);
        acc[10].fma_add(t2, y1);
        acc[11].fma_add(t2, y2);
        acc[12].fma_add(t3, y0);
        acc[13].fma_add(t3, y1);
        acc[14].fma_add(t3, y2);
        acc[15].fma_add(t3, y3);
        acc[16].fma_add(t4, y0);
        acc[17].fma_add(t4, y1);
        acc[18].fma_add(t4, y2);
        acc[19].fma_add(t4, y3);
        acc[20].fma_add(t4, y4);

        if constexpr (ADJ) {
            // log p(y_i) in nats (the same value in every lane of the group)
            const float lse = (lmax + __log2f(den)) * 0.69314718056f;
            accll.add(w * lse);
            // u = L^-T z restricted to the two directional coordinates (scaled by
            // log2(e)/2, removed in FP64 by the gradient assembly)
            const float u0 = fmaf(P[12], z0, fmaf(P[13], z1, fmaf(P[15], z2, fmaf(P[18], z3, P[22] * z4))));
            const float u1 = fmaf(P[14], z1, fmaf(P[16], z2, fmaf(P[19], z3, P[23] * z4)));
            // d nu / d delta_j: nu = f(z') (x', y'); along delta_j the frame turns so that
            // dz' = (x', y')_j, dx' = -[j==0] z' + phi_j y', dy' = -[j==1] z' - phi_j x'
            const float rs = __builtin_amdgcn_rsqf(fmaf(xr, xr, yr * yr));
            const float fp = dtheta_over_sin_dz(zr, rs);
            const float ph0 = P[28], ph1 = P[29];
            const float dz0 = xr, dz1 = yr;
            const float dx0 = fmaf(ph0, yr, -zr), dx1 = ph1 * yr;
            const float dy0 = -ph0 * xr, dy1 = fmaf(-ph1, xr, -zr);
            const float D00 = fmaf(fp * dz0, xr, f * dx0), D01 = fmaf(fp * dz1, xr, f * dx1);
            const float D10 = fmaf(fp * dz0, yr, f * dy0), D11 = fmaf(fp * dz1, yr, f * dy1);
            acc[NS - 2].add(wr * fmaf(D00, u0, D10 * u1));
            acc[NS - 1].add(wr * fmaf(D01, u0, D11 * u1));
        }
    };
    auto fold_all = [&]() {
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[s].fold();
        accll.fold();
    };

    // two steps per trip with alternating prefetch registers (no register copies)
    uint32_t i = (uint32_t)(wave * S + slot);
    SampleRegs a{}, b{};
    if (steps > 0) a = load_sample(ch, min(i, last));
    int64_t it = 0;
    for (; it + 1 < steps; it += 2) {
        b = load_sample(ch, min(i + ustride, last));
        body(a, i <= last);
        i += ustride;
        a = load_sample(ch, min(i + ustride, last));
        body(b, i <= last);
        i += ustride;
        if (((it + 2) % kFoldEvery) == 0) fold_all();
    }
    if (it < steps) body(a, i <= last);

    double v[NR];
#pragma unroll
    for (int s = 0; s < NS; ++s) v[s] = acc[s].total();
    double W, M, neg;
    weight_pass(smp + 6 * N, s0, s1, W, M, neg);
    v[NS] = slot == 0 ? W : 0.0;
    v[NS + 1] = slot == 0 ? M : 0.0;
    v[NS + 2] = slot == 0 ? neg : 0.0;
    if constexpr (ADJ) v[NS + 3] = accll.total();
    // sum over the sample slots (lanes with the same component), fixed butterfly order
#pragma unroll
    for (int o = G; o < 64; o <<= 1) {
#pragma unroll
        for (int s = 0; s < NR; ++s) v[s] += __shfl_xor(v[s], o);
    }
    if (lane < G) {
#pragma unroll
        for (int s = 0; s < NR; ++s) lds[(wave * NR + s) * G + comp] = v[s];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < NR * G; idx += blockDim.x) {
        const int s = idx / G, k = idx % G;
        double tot = 0.0;
        for (int wv = 0; wv < nwaves; ++wv) tot += lds[(wv * NR + s) * G + k];
        if (s < NS) {
            if (k < K) part[s * K + k] = tot;
        } else if (k == 0) {
            part[NS * K + (s - NS)] = tot;
        }
    }
}

}  // namespace sdmm
