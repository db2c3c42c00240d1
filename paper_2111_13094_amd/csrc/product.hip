// product.hip -- product sampling of a conditioned radiance mixture with a conditioned BSDF
// mixture on gfx950 (Dodik et al., arXiv 2111.13094, Sec. 3.4; the pruning to the two
// heaviest BSDF components of Sec. 4.1).
//
// Per query, in one group of G lanes (lane k = radiance component k, and lane b = BSDF
// component b while the BSDF model is conditioned):
//   1. both mixtures conditioned on their inputs (radiance: the position; BSDF: its three
//      inputs), weights by a DPP log-sum-exp;
//   2. the two BSDF components of largest weight (lowest index on ties) by two group
//      maxima; every BSDF lane rotates its own component to world (frame rows F t1, F t2,
//      F mu_b, in which offset and covariance keep their local values) and forms its
//      centre exp(m) and exp-map Jacobian; the two kept ones are broadcast;
//   3. lane k forms its two pairs: the BSDF component moved into the tangent space of
//      mu_k (centre a = log_mu_k(centre), covariance J S J^T with J the log-map Jacobian
//      at the centre times the exp-map Jacobian), and the product of the two 2-D
//      Gaussians: log2-weight, mean c, Cholesky factor of C and its scaled inverse;
//   4. draws: pair by a group prefix sum over lanes (pair order 2k + j), Box-Muller,
//      nu = c + L_C z, cut-locus discard, exp map; the pdf of the normalised product
//      mixture at the drawn direction (one log map per lane, two 2-D quadratic forms).
#include <algorithm>

#include "common.hpp"
#include "query_common.hpp"
#include "timing.hpp"

namespace sdmm {

constexpr float kLog2eF = 1.4426950408889634f;
constexpr float kLog2TwoPi = 2.6514961294723187f;  // log2(2 pi)
constexpr float kHalfLog2e = 0.72134752044448170f;

// A BSDF component rotated to world and prepared for the pairs: its offset and
// covariance in the rotated frame, its centre exp(m) and the world-space exp-map
// Jacobian D = d exp / d nu at m (3 x 2), and its log2 weight.
struct BsdfWorld {
    float m0, m1, s00, s01, s11;
    float cx, cy, cz;
    float d[6];  // D row-major: d[2 i + c]
    float lw;
};

// rotates the component of table row TB (conditioned offset bm0, bm1) by F (row-major,
// world = F local) and prepares it. The rotated frame rows F t1, F t2, F mu are an
// orthonormal frame about the rotated mean in which the offset and the covariance keep
// their local values, so the component needs no frame of its own.
__device__ __forceinline__ BsdfWorld rotate_bsdf(const float* TB, float bm0, float bm1, const float* F, float lw)
{
    BsdfWorld o;
    float Rw[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int i = 0; i < 3; ++i)
            Rw[3 * r + i] = fmaf(F[3 * i], TB[3 * r], fmaf(F[3 * i + 1], TB[3 * r + 1], F[3 * i + 2] * TB[3 * r + 2]));
    o.m0 = bm0;
    o.m1 = bm1;
    // S = L' L'^T
    const float l0 = TB[24], l1 = TB[25], l2 = TB[26];
    o.s00 = l0 * l0;
    o.s01 = l0 * l1;
    o.s11 = fmaf(l1, l1, l2 * l2);
    // centre and exp-map Jacobian at m: w = Rw^T v, v = (nu sinc r, cos r),
    // dv/dnu = [[s + n0^2 c, n0 n1 c], [n0 n1 c, s + n1^2 c], [-n0 s, -n1 s]]
    const float r2 = fmaf(o.m0, o.m0, o.m1 * o.m1);
    const float r = __builtin_amdgcn_sqrtf(r2);
    const float rev = r * 0.15915494309189535f;
    const float sr = __builtin_amdgcn_sinf(rev), cr = __builtin_amdgcn_cosf(rev);
    const bool small = r < 1e-2f;
    const float sc = small ? fmaf(-r2, 1.0f / 6.0f, 1.0f) : sr * __builtin_amdgcn_rcpf(r);
    const float c = small ? fmaf(r2, 1.0f / 30.0f, -1.0f / 3.0f) : (cr - sc) * __builtin_amdgcn_rcpf(r2);
    const float v0 = o.m0 * sc, v1 = o.m1 * sc;
    o.cx = fmaf(Rw[0], v0, fmaf(Rw[3], v1, Rw[6] * cr));
    o.cy = fmaf(Rw[1], v0, fmaf(Rw[4], v1, Rw[7] * cr));
    o.cz = fmaf(Rw[2], v0, fmaf(Rw[5], v1, Rw[8] * cr));
    const float M00 = fmaf(o.m0 * o.m0, c, sc), M01 = o.m0 * o.m1 * c, M11 = fmaf(o.m1 * o.m1, c, sc);
    const float M20 = -o.m0 * sc, M21 = -o.m1 * sc;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        o.d[2 * i] = fmaf(Rw[i], M00, fmaf(Rw[3 + i], M01, Rw[6 + i] * M20));
        o.d[2 * i + 1] = fmaf(Rw[i], M01, fmaf(Rw[3 + i], M11, Rw[6 + i] * M21));
    }
    o.lw = lw;
    return o;
}

__device__ __forceinline__ BsdfWorld shfl_bsdf(const BsdfWorld& v, int src)
{
    BsdfWorld o;
    o.m0 = __shfl(v.m0, src);
    o.m1 = __shfl(v.m1, src);
    o.s00 = __shfl(v.s00, src);
    o.s01 = __shfl(v.s01, src);
    o.s11 = __shfl(v.s11, src);
    o.cx = __shfl(v.cx, src);
    o.cy = __shfl(v.cy, src);
    o.cz = __shfl(v.cz, src);
#pragma unroll
    for (int i = 0; i < 6; ++i) o.d[i] = __shfl(v.d[i], src);
    o.lw = __shfl(v.lw, src);
    return o;
}

// one product pair in the tangent space of the radiance component (frame R, conditioned
// offset m, covariance from the table's L')
struct Pair {
    float l;             // log2 weight (-inf: empty)
    float c0, c1;        // mean
    float i0, i1, i2;    // inverse of the Cholesky factor of C times sqrt(log2(e) / 2)
    float nrm;           // -log2(2 pi det L_C)
};

constexpr float kKap = 0.84932180028801904f;   // sqrt(log2(e) / 2)
constexpr float kIKap = 1.1774100225154747f;   // its reciprocal

// the Cholesky factor L = (l0; l1 l2) of a pair's C from its scaled inverse (the draws)
__device__ __forceinline__ void pair_factor(float i0, float i1, float i2, float& l0, float& l1, float& l2)
{
    l0 = kKap * __builtin_amdgcn_rcpf(i0);
    l2 = kKap * __builtin_amdgcn_rcpf(i2);
    l1 = -i1 * l0 * l2 * kIKap;
}

__device__ __forceinline__ Pair make_pair(const float* R, float lwk, float m0, float m1, float a00, float a01,
                                          float a11, const BsdfWorld& b)
{
    Pair p;
    p.l = -INFINITY;
    p.c0 = p.c1 = 0.0f;
    p.i0 = p.i2 = 1.0f;
    p.i1 = 0.0f;
    p.nrm = 0.0f;
    // centre in the frame of mu_k and the log-map Jacobian there:
    // nu = f (x, y), d f / d x = x g, d f / d y = y g, d f / d z = -1, g = (z - f) / s^2
    const float px = fmaf(R[0], b.cx, fmaf(R[1], b.cy, fmaf(R[2], b.cz, 1e-18f)));
    const float py = fmaf(R[3], b.cx, fmaf(R[4], b.cy, R[5] * b.cz));
    const float pz = fmaf(R[6], b.cx, fmaf(R[7], b.cy, R[8] * b.cz));
    float a0, a1;
    const float f = log_map_f32_offset(px, py, pz, a0, a1);
    const float s2 = fmaf(px, px, py * py);
    const float g = s2 > 1e-6f ? (pz - f) * __builtin_amdgcn_rcpf(s2) : -2.0f / 3.0f;
    const float J00 = fmaf(px * px, g, f), J01 = px * py * g, J02 = -px;
    const float J11 = fmaf(py * py, g, f), J12 = -py;
    // E = R D (3 x 2), then J = Jl E (2 x 2)
    float E[6];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        E[2 * i] = fmaf(R[3 * i], b.d[0], fmaf(R[3 * i + 1], b.d[2], R[3 * i + 2] * b.d[4]));
        E[2 * i + 1] = fmaf(R[3 * i], b.d[1], fmaf(R[3 * i + 1], b.d[3], R[3 * i + 2] * b.d[5]));
    }
    const float j00 = fmaf(J00, E[0], fmaf(J01, E[2], J02 * E[4]));
    const float j01 = fmaf(J00, E[1], fmaf(J01, E[3], J02 * E[5]));
    const float j10 = fmaf(J01, E[0], fmaf(J11, E[2], J12 * E[4]));
    const float j11 = fmaf(J01, E[1], fmaf(J11, E[3], J12 * E[5]));
    // B = J S J^T
    const float u00 = fmaf(j00, b.s00, j01 * b.s01), u01 = fmaf(j00, b.s01, j01 * b.s11);
    const float u10 = fmaf(j10, b.s00, j11 * b.s01), u11 = fmaf(j10, b.s01, j11 * b.s11);
    const float b00 = fmaf(u00, j00, u01 * j01), b01 = fmaf(u10, j00, u11 * j01), b11 = fmaf(u10, j10, u11 * j11);
    // S = A + B and the weight N(m; a, S)
    const float S00 = a00 + b00, S01 = a01 + b01, S11 = a11 + b11;
    const float det = fmaf(S00, S11, -S01 * S01);
    const bool ok = det > 0.0f && isfinite(lwk) && isfinite(b.lw) && isfinite(det);
    const float idet = __builtin_amdgcn_rcpf(det);
    const float si00 = S11 * idet, si01 = -S01 * idet, si11 = S00 * idet;
    const float d0 = m0 - a0, d1 = m1 - a1;
    const float q = fmaf(d0, fmaf(si00, d0, si01 * d1), d1 * fmaf(si01, d0, si11 * d1));
    // C = A S^-1 B and c = m - A S^-1 (m - a) (equal to B S^-1 m + A S^-1 a, since
    // A S^-1 + B S^-1 = I)
    const float as00 = fmaf(a00, si00, a01 * si01), as01 = fmaf(a00, si01, a01 * si11);
    const float as10 = fmaf(a01, si00, a11 * si01), as11 = fmaf(a01, si01, a11 * si11);
    const float C00 = fmaf(as00, b00, as01 * b01);
    const float C01 = 0.5f * (fmaf(as00, b01, as01 * b11) + fmaf(as10, b00, as11 * b01));
    const float C11 = fmaf(as10, b01, as11 * b11);
    const float rc = __builtin_amdgcn_rcpf(C00);
    const float L2s = fmaf(-C01, C01 * rc, C11);  // the factor's last pivot squared
    if (!(ok && C00 > 0.0f && L2s > 0.0f)) return p;
    p.c0 = m0 - fmaf(as00, d0, as01 * d1);
    p.c1 = m1 - fmaf(as10, d0, as11 * d1);
    // inverse factor from the pivots' reciprocal square roots: L0 = sqrt(C00),
    // L1 = C01 / L0, L2 = sqrt(L2s); (L^-1)_10 = -L1 / (L0 L2) = -(C01 / C00) / L2
    const float r0 = __builtin_amdgcn_rsqf(C00), r2 = __builtin_amdgcn_rsqf(L2s);
    p.i0 = kKap * r0;
    p.i2 = kKap * r2;
    p.i1 = -C01 * rc * p.i2;
    p.nrm = __builtin_amdgcn_logf(r0 * r2) - kLog2TwoPi;
    p.l = lwk + b.lw - kHalfLog2e * q - kLog2TwoPi - 0.5f * __builtin_amdgcn_logf(det);
    return p;
}

// P N(nu; c, C) at a lane's tangent coordinates
__device__ __forceinline__ float pair_density(const Pair& p, float P, float n0, float n1)
{
    const float d0 = n0 - p.c0, d1 = n1 - p.c1;
    const float z0 = p.i0 * d0, z1 = fmaf(p.i1, d0, p.i2 * d1);
    return P * __builtin_amdgcn_exp2f(p.nrm - fmaf(z0, z0, z1 * z1));
}

// Per-query state after the set-up: lane k's frame and two pairs with probabilities.
struct ProductQuery {
    float R[9];
    Pair p0, p1;
    float P0, P1;
    bool any;  // some pair has weight
};

// Set-up of one query (steps 1-3). Lanes of a group must all call it.
template <int G>
__device__ __forceinline__ void product_setup(const float* __restrict__ table, int C, int K,
                                              const float* __restrict__ btable, int CB, int Kb, int qc, int bc,
                                              bool inq, float x0, float x1, float x2, float y0, float y1, float y2,
                                              const float* F, ProductQuery& Qy)
{
    const int lane = threadIdx.x & 63, comp = lane % G, base = lane - comp;
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << base);
    const bool usable = inq && qc >= 0 && qc < C && bc >= 0 && bc < CB;
    // radiance conditioning
    float T[kCond];
    load_row(table_row(table, qc, K, comp, usable), K, T);
    float m0, m1;
    float lw = cond_component(T, x0, x1, x2, m0, m1);
    if (comp >= K || !usable) lw = -INFINITY;
    float wk_unused;
    const float lwk = cond_log_weight<G>(lw, wk_unused);
#pragma unroll
    for (int i = 0; i < 9; ++i) Qy.R[i] = T[i];
    const float l0 = T[24], l1 = T[25], l2 = T[26];
    const float a00 = l0 * l0, a01 = l0 * l1, a11 = fmaf(l1, l1, l2 * l2);
    // BSDF conditioning (lane b = component b), its weights, and the two heaviest
    float TB[kCond];
    load_row(table_row(btable, bc, Kb, comp, usable), Kb, TB);
    float bm0, bm1;
    float lb = cond_component(TB, y0, y1, y2, bm0, bm1);
    if (comp >= Kb || !usable) lb = -INFINITY;
    float wb;
    const float lwb = cond_log_weight<G>(lb, wb);
    const float w1 = group_max<G>(wb);
    const uint64_t h0 = __ballot(comp < Kb && wb > 0.0f && wb == w1) & gmask;
    const int s0 = h0 ? __builtin_ctzll(h0) - base : -1;
    const float wb2 = (comp == s0) ? -1.0f : wb;
    const float w2 = group_max<G>(wb2);
    const uint64_t h1 = __ballot(comp < Kb && wb2 > 0.0f && wb2 == w2) & gmask;
    const int s1 = h1 ? __builtin_ctzll(h1) - base : -1;
    const BsdfWorld mine = rotate_bsdf(TB, bm0, bm1, F, lwb);
    BsdfWorld b0 = shfl_bsdf(mine, base + (s0 < 0 ? 0 : s0));
    BsdfWorld b1 = shfl_bsdf(mine, base + (s1 < 0 ? 0 : s1));
    if (s0 < 0) b0.lw = -INFINITY;
    if (s1 < 0) b1.lw = -INFINITY;
    // pairs and their probabilities
    Qy.p0 = make_pair(Qy.R, lwk, m0, m1, a00, a01, a11, b0);
    Qy.p1 = make_pair(Qy.R, lwk, m0, m1, a00, a01, a11, b1);
    if (comp >= K) Qy.p0.l = Qy.p1.l = -INFINITY;
    // pair probabilities: exp2 of the log2 weights normalised over the 2K pairs; a group
    // whose sum leaves [2^-100, 2^100] takes the group maximum first
    float e0 = __builtin_amdgcn_exp2f(Qy.p0.l), e1 = __builtin_amdgcn_exp2f(Qy.p1.l);
    float tot = group_sum<G>(e0 + e1);
    const bool out = !(tot >= 0x1p-100f && tot <= 0x1p100f);
    Qy.any = true;
    if (__ballot(out)) {
        const float lm = group_max<G>(fmaxf(Qy.p0.l, Qy.p1.l));
        const bool any = lm != -INFINITY;
        const float f0 = any ? __builtin_amdgcn_exp2f(Qy.p0.l - lm) : 0.0f;
        const float f1 = any ? __builtin_amdgcn_exp2f(Qy.p1.l - lm) : 0.0f;
        const float t2 = group_sum<G>(f0 + f1);
        e0 = out ? f0 : e0;
        e1 = out ? f1 : e1;
        tot = out ? t2 : tot;
        Qy.any = out ? any : true;
    }
    const float itot = tot > 0.0f ? __builtin_amdgcn_rcpf(tot) : 0.0f;
    Qy.P0 = e0 * itot;
    Qy.P1 = e1 * itot;
}

// the lane's share of the density of the normalised product mixture at a world direction
// (step 4): its component's two pairs, 0 past K and at the cut locus
__device__ __forceinline__ float product_density_lane(const ProductQuery& Qy, int K, int comp, float wx, float wy,
                                                      float wz)
{
    // the 1e-18 offset of the log map rides on the rotation's first row
    const float xr = fmaf(Qy.R[0], wx, fmaf(Qy.R[1], wy, fmaf(Qy.R[2], wz, 1e-18f)));
    const float yr = fmaf(Qy.R[3], wx, fmaf(Qy.R[4], wy, Qy.R[5] * wz));
    const float zr = fmaf(Qy.R[6], wx, fmaf(Qy.R[7], wy, Qy.R[8] * wz));
    float n0, n1;
    const float f = log_map_f32_offset(xr, yr, zr, n0, n1);
    const float r2 = fmaf(n0, n0, n1 * n1);
    const float v = pair_density(Qy.p0, Qy.P0, n0, n1) + pair_density(Qy.p1, Qy.P1, n0, n1);
    return (comp < K && r2 < kCutSq) ? v * f : 0.0f;
}

// density of the normalised product mixture at a world direction (all lanes of the group)
template <int G>
__device__ __forceinline__ float product_density(const ProductQuery& Qy, int K, float wx, float wy, float wz)
{
    return group_sum<G>(product_density_lane(Qy, K, (threadIdx.x & 63) % G, wx, wy, wz));
}

__device__ __forceinline__ void load_frame(const float* __restrict__ frames, int64_t nq, int64_t q, float F[9])
{
#pragma unroll
    for (int i = 0; i < 9; ++i) F[i] = frames[i * nq + q];
}

// Draws (step 4), G at a time, draw t0 + c by lane c of the query's group: the group picks
// every draw's pair against the query's pair CDF (one group prefix sum per query; pair
// 2k + j, lowest index on ties), lane c gathers its pair (the radiance frame and the
// pair's mean and factor) from the lane that holds it and forms the candidate, and the
// group then evaluates the normalised product density at each draw's direction.
template <int G>
__global__ __launch_bounds__(256) void product_sample_kernel(
    const float* __restrict__ table, int C, int K, const float* __restrict__ qpos, const int32_t* __restrict__ qcell,
    const float* __restrict__ btable, int CB, int Kb, const float* __restrict__ bpar,
    const int32_t* __restrict__ bcell, const float* __restrict__ frames, int64_t nq, int ns,
    const float* __restrict__ uniforms, uint64_t seed, float* __restrict__ dirs_out, float* __restrict__ pdf_out,
    uint8_t* __restrict__ valid_out, int32_t* __restrict__ pair_out)
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
        float F[9];
        load_frame(frames, nq, qq, F);
        ProductQuery Qy;
        product_setup<G>(table, C, K, btable, CB, Kb, qcell[qq], bcell[qq], inq, qpos[qq], qpos[nq + qq],
                         qpos[2 * nq + qq], bpar[qq], bpar[nq + qq], bpar[2 * nq + qq], F, Qy);
        const float s = Qy.P0 + Qy.P1;
        const float cdf = group_inclusive_scan<G>(s);
        const bool cand = comp < K && Qy.any;
        const uint64_t pos = __ballot(cand && s > 0.0f) & gmask;
        const int last_pos = pos ? 63 - __builtin_clzll(pos) - base : -1;
        const int j_last = __shfl(Qy.P1 > 0.0f ? 1 : 0, base + (last_pos < 0 ? 0 : last_pos));
        for (int t0 = 0; t0 < ns; t0 += G) {
            float ul0 = 0.0f, ul1 = 0.0f, ul2 = 0.0f;
            if (t0 + comp < ns) draw_uniforms(uniforms, nd, qq * ns + t0 + comp, seed, ul0, ul1, ul2);
            const int tn = min(G, ns - t0);  // wave-uniform
            // pair of every draw of the batch, four at a time (a draw past tn repeats the
            // last one and is not kept); lane c keeps the one of draw t0 + c
            int sel = -1, j = 0;
            for (int tt = 0; tt < tn; tt += 4) {
                float u0[4];
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) u0[k4] = __shfl(ul0, base + min(tt + k4, tn - 1));
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    const uint64_t hit = __ballot(cand && u0[k4] < cdf) & gmask;
                    const int s_hit = hit ? __builtin_ctzll(hit) - base : 0;
                    const int jh = (u0[k4] < (cdf - s) + Qy.P0 && Qy.P0 > 0.0f) || !(Qy.P1 > 0.0f) ? 0 : 1;
                    const int j_hit = __shfl(jh, base + s_hit);
                    const bool mine = comp == tt + k4;
                    sel = mine ? (hit ? s_hit : last_pos) : sel;
                    j = mine ? (hit ? j_hit : j_last) : j;
                }
            }
            const int src = base + (sel < 0 ? 0 : sel);
            float R[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) R[i] = __shfl(Qy.R[i], src);
            // both pairs' means and scaled inverse factors from the lane that holds them, then
            // this draw's pair (j) and its factor
            const float a0 = __shfl(Qy.p0.i0, src), a1 = __shfl(Qy.p0.i1, src), a2 = __shfl(Qy.p0.i2, src);
            const float ac0 = __shfl(Qy.p0.c0, src), ac1 = __shfl(Qy.p0.c1, src);
            const float b0 = __shfl(Qy.p1.i0, src), b1 = __shfl(Qy.p1.i1, src), b2 = __shfl(Qy.p1.i2, src);
            const float bc0 = __shfl(Qy.p1.c0, src), bc1 = __shfl(Qy.p1.c1, src);
            const float c0 = j ? bc0 : ac0, c1 = j ? bc1 : ac1;
            float l0, l1, l2;
            pair_factor(j ? b0 : a0, j ? b1 : a1, j ? b2 : a2, l0, l1, l2);
            float w[3];
            const int ok = draw_candidate(R, l0, l1, l2, c0, c1, ul1, ul2, w);
            const int valid = sel >= 0 && ok;
            float pdf = 0.0f;
            for (int tt = 0; tt < tn; tt += 4) {
                float v[4];
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    const int from = base + min(tt + k4, tn - 1);
                    v[k4] = product_density_lane(Qy, K, comp, __shfl(w[0], from), __shfl(w[1], from),
                                                 __shfl(w[2], from));
                }
                if constexpr (G == 16) {
                    // lane comp ends with the sum for draw tt + (comp & 3)
                    const float p = group_sum4_row16(v);
                    pdf = (comp >> 2) == (tt >> 2) ? p : pdf;
                } else {
#pragma unroll
                    for (int k4 = 0; k4 < 4; ++k4) {
                        const float p = group_sum<G>(v[k4]);
                        pdf = comp == tt + k4 ? p : pdf;
                    }
                }
            }
            if (inq && comp < tn) {
                const int64_t d = qq * ns + t0 + comp;
                dirs_out[d] = valid ? w[0] : 0.0f;
                dirs_out[nd + d] = valid ? w[1] : 0.0f;
                dirs_out[2 * nd + d] = valid ? w[2] : 0.0f;
                pdf_out[d] = valid ? pdf : 0.0f;
                valid_out[d] = (uint8_t)valid;
                if (pair_out) pair_out[d] = sel >= 0 ? 2 * sel + j : -1;
            }
        }
    }
}

// The same set-up, draws and pdf as product_sample_kernel in three wave-local phases over
// QB = S * nqr queries (nqr <= 2 rounds of S queries, QB * ns <= 64 draws), as in the
// fused query kernel:
//   A. set-up, lane = (query slot, component), per round (steps 1-3): the lane's two
//      pairs (mean, scaled inverse factor, normaliser, probability) and the pair CDF
//      into LDS, with each query's cell, last component of positive weight and its pair;
//   B. the draws, one per lane: uniforms, the component by the first CDF entry above u0
//      and the pair within it, then the candidate from the pair's mean and the factor
//      taken back from its inverse, in the frame of the component's table row;
//   C. the pdf, lane = (query slot, component) again: every draw of the query over the
//      lane's two pairs, four at a time.
// Phase B runs on QB * ns lanes where product_sample_kernel draws on ns of each query's G
// lanes. Pair choices are the same as there; a candidate differs by the rounding of the
// recovered factor.
constexpr int kProdWpb = 2;   // waves per work group (LDS: about 8.6 KB per wave)
constexpr int kProdRounds = 2;
constexpr int kPairF = 7;     // per pair: c0, c1, i0, i1, i2, nrm, probability

template <int G>
__global__ __launch_bounds__(64 * kProdWpb) void product_sample_lanes_kernel(
    const float* __restrict__ table, int C, int K, const float* __restrict__ qpos, const int32_t* __restrict__ qcell,
    const float* __restrict__ btable, int CB, int Kb, const float* __restrict__ bpar,
    const int32_t* __restrict__ bcell, const float* __restrict__ frames, int64_t nq, int ns, int nqr,
    const float* __restrict__ uniforms, uint64_t seed, float* __restrict__ dirs_out, float* __restrict__ pdf_out,
    uint8_t* __restrict__ valid_out, int32_t* __restrict__ pair_out)
{
    constexpr int S = 64 / G, QBMAX = kProdRounds * S, WPB = kProdWpb;
    // per wave: the pair CDF of its queries (-inf on lanes no draw may pick), each lane's
    // two pairs by field ([round][field][lane]), each query's cell (-1: none), last
    // component of positive weight and the pair used past it, and the draws' directions
    // with their validity in .w
    __shared__ __align__(16) float cdf_s[WPB][QBMAX][G];
    __shared__ float pd_s[WPB][kProdRounds][2 * kPairF][64];
    __shared__ int last_s[WPB][QBMAX], jl_s[WPB][QBMAX], cell_s[WPB][QBMAX];
    __shared__ float4 w_s[WPB][64];
    const int lane = threadIdx.x & 63, comp = lane % G, slot = lane / G, base = lane - comp;
    const int wv = threadIdx.x >> 6;
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << base);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t nd = nq * ns;
    const int QB = S * nqr;
    for (int64_t qb = wave * QB; qb < nq; qb += nwaves * QB) {
        // A: set-up
        for (int r = 0; r < nqr; ++r) {
            const int qi = r * S + slot;
            const int64_t q = qb + qi;
            const bool inq = q < nq;
            const int64_t qq = inq ? q : 0;
            // channel strides (and below the generator's round keys) are formed where they
            // are used, by scalar instructions, instead of being held across the loop in
            // scalar registers that spill
            int64_t nqo = nq;
            asm volatile("" : "+s"(nqo));
            float F[9];
            load_frame(frames, nqo, qq, F);
            const int qc = qcell[qq], bc = bcell[qq];
            ProductQuery Qy;
            product_setup<G>(table, C, K, btable, CB, Kb, qc, bc, inq, qpos[qq], qpos[nqo + qq], qpos[2 * nqo + qq],
                             bpar[qq], bpar[nqo + qq], bpar[2 * nqo + qq], F, Qy);
            const float s = Qy.P0 + Qy.P1;
            const float cdf = group_inclusive_scan<G>(s);
            const bool cand = comp < K && Qy.any;
            const uint64_t pos = __ballot(cand && s > 0.0f) & gmask;
            const int last_pos = pos ? 63 - __builtin_clzll(pos) - base : -1;
            const int j_last = __shfl(Qy.P1 > 0.0f ? 1 : 0, base + (last_pos < 0 ? 0 : last_pos));
            cdf_s[wv][qi][comp] = cand ? cdf : -INFINITY;
            float* pd = &pd_s[wv][r][0][lane];
            pd[0 * 64] = Qy.p0.c0;
            pd[1 * 64] = Qy.p0.c1;
            pd[2 * 64] = Qy.p0.i0;
            pd[3 * 64] = Qy.p0.i1;
            pd[4 * 64] = Qy.p0.i2;
            pd[5 * 64] = Qy.p0.nrm;
            pd[6 * 64] = Qy.P0;
            pd[7 * 64] = Qy.p1.c0;
            pd[8 * 64] = Qy.p1.c1;
            pd[9 * 64] = Qy.p1.i0;
            pd[10 * 64] = Qy.p1.i1;
            pd[11 * 64] = Qy.p1.i2;
            pd[12 * 64] = Qy.p1.nrm;
            pd[13 * 64] = Qy.P1;
            if (comp == 0) {
                last_s[wv][qi] = last_pos;
                jl_s[wv][qi] = j_last;
                cell_s[wv][qi] = (inq && qc >= 0 && qc < C && bc >= 0 && bc < CB) ? qc : -1;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // this wave's LDS writes are done
        // B: one draw per lane
        {
            const int qi = lane / ns, t = lane % ns;
            const int64_t q = qb + qi;
            const bool act = qi < QB && q < nq;
            const int64_t d = act ? q * ns + t : 0;
            uint64_t key = seed;
            int64_t ndo = nd;
            asm volatile("" : "+s"(key), "+s"(ndo));
            float u0, u1, u2;
            draw_uniforms(uniforms, ndo, d, key, u0, u1, u2);
            const int qis = act ? qi : 0;
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
            const bool hit = first >= 0;
            const int sel = hit ? first : last_s[wv][qis];
            const int sk = sel < 0 ? 0 : sel;
            const float* pd = &pd_s[wv][qis / S][0][(qis % S) * G + sk];
            // the pair within the component: the first unless u0 lies past its share of the CDF
            const float P0 = pd[6 * 64], P1 = pd[13 * 64];
            const float cdfv = cdf_s[wv][qis][sk];
            const int jh = (u0 < (cdfv - (P0 + P1)) + P0 && P0 > 0.0f) || !(P1 > 0.0f) ? 0 : 1;
            const int j = hit ? jh : jl_s[wv][qis];
            const float* pj = pd + (j ? kPairF * 64 : 0);
            const float c0 = pj[0], c1 = pj[64], i0 = pj[2 * 64], i1 = pj[3 * 64], i2 = pj[4 * 64];
            float L0, L1, L2;
            pair_factor(i0, i1, i2, L0, L1, L2);
            const int qc = cell_s[wv][qis];
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
            float w[3];
            const int ok = draw_candidate(R, L0, L1, L2, c0, c1, u1, u2, w);
            const int valid = act && sel >= 0 && ok;
            w_s[wv][lane] = make_float4(w[0], w[1], w[2], valid ? 1.0f : 0.0f);
            if (act) {  // the pass's draws are contiguous: d = qb * ns + lane
                dirs_out[d] = valid ? w[0] : 0.0f;
                dirs_out[ndo + d] = valid ? w[1] : 0.0f;
                dirs_out[2 * ndo + d] = valid ? w[2] : 0.0f;
                valid_out[d] = (uint8_t)valid;
                if (pair_out) pair_out[d] = sel >= 0 ? 2 * sel + j : -1;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        // C: the pdf of every draw over the lane's two pairs, outputs
        for (int r = 0; r < nqr; ++r) {
            const int qi = r * S + slot;
            const int64_t q = qb + qi;
            const bool inq = q < nq;
            const int qc = cell_s[wv][qi];
            ProductQuery Qy;
            const float4* row = reinterpret_cast<const float4*>(table_row(table, qc, K, comp, qc >= 0));
            float R[12];
#pragma unroll
            for (int c4 = 0; c4 < 3; ++c4) {
                const float4 v = row[(int64_t)c4 * K];
                R[4 * c4] = v.x;
                R[4 * c4 + 1] = v.y;
                R[4 * c4 + 2] = v.z;
                R[4 * c4 + 3] = v.w;
            }
#pragma unroll
            for (int i = 0; i < 9; ++i) Qy.R[i] = R[i];
            const float* pd = &pd_s[wv][r][0][lane];
            Qy.p0.c0 = pd[0 * 64];
            Qy.p0.c1 = pd[1 * 64];
            Qy.p0.i0 = pd[2 * 64];
            Qy.p0.i1 = pd[3 * 64];
            Qy.p0.i2 = pd[4 * 64];
            Qy.p0.nrm = pd[5 * 64];
            Qy.P0 = pd[6 * 64];
            Qy.p1.c0 = pd[7 * 64];
            Qy.p1.c1 = pd[8 * 64];
            Qy.p1.i0 = pd[9 * 64];
            Qy.p1.i1 = pd[10 * 64];
            Qy.p1.i2 = pd[11 * 64];
            Qy.p1.nrm = pd[12 * 64];
            Qy.P1 = pd[13 * 64];
            float pdf = 0.0f;
            for (int tt = 0; tt < ns; tt += 4) {  // wave-uniform
                const float4* wq = &w_s[wv][qi * ns + tt];
                float v[4];
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    const float4 wd = wq[min(k4, ns - 1 - tt)];  // past the last draw: repeat it
                    v[k4] = product_density_lane(Qy, K, comp, wd.x, wd.y, wd.z);
                }
                if constexpr (G == 16) {
                    // lane comp ends with the sum for draw tt + (comp & 3)
                    const float p = group_sum4_row16(v);
                    pdf = (comp >> 2) == (tt >> 2) ? p : pdf;
                } else {
#pragma unroll
                    for (int k4 = 0; k4 < 4; ++k4) {
                        const float p = group_sum<G>(v[k4]);
                        pdf = comp == tt + k4 ? p : pdf;
                    }
                }
            }
            if (inq && comp < ns) pdf_out[q * ns + comp] = w_s[wv][qi * ns + comp].w != 0.0f ? pdf : 0.0f;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // before the next pass overwrites
    }
}

template <int G>
__global__ __launch_bounds__(256) void product_pdf_kernel(
    const float* __restrict__ table, int C, int K, const float* __restrict__ qpos, const int32_t* __restrict__ qcell,
    const float* __restrict__ btable, int CB, int Kb, const float* __restrict__ bpar,
    const int32_t* __restrict__ bcell, const float* __restrict__ frames, int64_t nq, int nd,
    const float* __restrict__ dirs, float* __restrict__ pdf_out)
{
    constexpr int S = 64 / G;
    const int lane = threadIdx.x & 63, comp = lane % G, slot = lane / G;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t np = nq * nd;
    for (int64_t q0 = wave * S; q0 < nq; q0 += nwaves * S) {
        const int64_t q = q0 + slot;
        const bool inq = q < nq;
        const int64_t qq = inq ? q : 0;
        float F[9];
        load_frame(frames, nq, qq, F);
        ProductQuery Qy;
        product_setup<G>(table, C, K, btable, CB, Kb, qcell[qq], bcell[qq], inq, qpos[qq], qpos[nq + qq],
                         qpos[2 * nq + qq], bpar[qq], bpar[nq + qq], bpar[2 * nq + qq], F, Qy);
        for (int t = 0; t < nd; ++t) {
            const int64_t p = qq * nd + t;
            const float v = product_density<G>(Qy, K, dirs[p], dirs[np + p], dirs[2 * np + p]);
            if (inq && comp == 0) pdf_out[p] = Qy.any ? v : 0.0f;
        }
    }
}

static int product_args_ok(const float* table, int32_t n_cells, int32_t K, const float* btable, int32_t n_bsdf,
                           int32_t Kb, int64_t nq, int32_t n)
{
    return table && btable && n_cells > 0 && n_bsdf > 0 && K >= 1 && K <= kMaxK && Kb >= 1 && Kb <= kMaxK &&
           nq >= 0 && n >= 0;
}

}  // namespace sdmm

using namespace sdmm;

extern "C" int sdmm_product_sample(const float* table, int32_t n_cells, int32_t K, const float* qpos,
                                   const int32_t* qcell, const float* btable, int32_t n_bsdf, int32_t Kb,
                                   const float* bpar, const int32_t* bcell, const float* frames, int64_t nq,
                                   int32_t ns, const float* uniforms, uint64_t seed, float* dirs_out,
                                   float* pdf_out, uint8_t* valid_out, int32_t* pair_out, void* stream)
{
    if (!product_args_ok(table, n_cells, K, btable, n_bsdf, Kb, nq, ns)) return SDMM_EINVAL;
    if (nq == 0 || ns == 0) return SDMM_OK;
    if (!qpos || !qcell || !bpar || !bcell || !frames || !dirs_out || !pdf_out || !valid_out) return SDMM_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int G = group_for(K > Kb ? K : Kb);
    ScopedTimer tm(SDMM_TIMER_PRODUCT, s);
    const int S = 64 / G;
    if (S * ns <= 64) {
        // the draws of up to two rounds of S queries share one pass of the draw phase
        const int nqr = std::max(1, std::min(kProdRounds, 64 / (S * ns)));
        SDMM_DISPATCH_G(G, (product_sample_lanes_kernel<g><<<grid_for(nq, S * nqr, kProdWpb), 64 * kProdWpb, 0, s>>>(
                               table, n_cells, K, qpos, qcell, btable, n_bsdf, Kb, bpar, bcell, frames, nq, ns, nqr,
                               uniforms, seed, dirs_out, pdf_out, valid_out, pair_out)));
    } else {
        SDMM_DISPATCH_G(G, (product_sample_kernel<g><<<grid_for(nq, 64 / g), 256, 0, s>>>(
                               table, n_cells, K, qpos, qcell, btable, n_bsdf, Kb, bpar, bcell, frames, nq, ns,
                               uniforms, seed, dirs_out, pdf_out, valid_out, pair_out)));
    }
    return check(hipGetLastError());
}

extern "C" int sdmm_product_pdf(const float* table, int32_t n_cells, int32_t K, const float* qpos,
                                const int32_t* qcell, const float* btable, int32_t n_bsdf, int32_t Kb,
                                const float* bpar, const int32_t* bcell, const float* frames, int64_t nq, int32_t nd,
                                const float* dirs, float* pdf_out, void* stream)
{
    if (!product_args_ok(table, n_cells, K, btable, n_bsdf, Kb, nq, nd)) return SDMM_EINVAL;
    if (nq == 0 || nd == 0) return SDMM_OK;
    if (!qpos || !qcell || !bpar || !bcell || !frames || !dirs || !pdf_out) return SDMM_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int G = group_for(K > Kb ? K : Kb);
    SDMM_DISPATCH_G(G, (product_pdf_kernel<g><<<grid_for(nq, 64 / g), 256, 0, s>>>(
                           table, n_cells, K, qpos, qcell, btable, n_bsdf, Kb, bpar, bcell, frames, nq, nd, dirs,
                           pdf_out)));
    return check(hipGetLastError());
}
