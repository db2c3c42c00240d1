// query_common.hpp -- pieces shared by the query kernels (conditioning, pdf, sampling)
// and the product-sampling kernels: the conditioning table layout, per-lane conditioning
// and exp map, the counter-based uniforms, the group prefix sum, table loads and the
// launch helpers.
#pragma once

#include "common.hpp"

namespace sdmm {

// conditioning table: per cell, the eight 16-byte chunks of its K components stored chunk
// by chunk ([cell][chunk][component][4 floats]), so that the lanes of a group, one
// component each, read one chunk of every component from contiguous memory. Per
// component (FP32):
//   0-8   R_mu rows (t1, t2, mu)           9-11  mu_x
//   12-17 Lxx^-1 * sqrt(log2(e)/2), packed   18-23 A = Sigma_nx Sigma_xx^-1 (2x3, row-major)
//   24-26 L' packed (chol of Sigma')         27-29 L'^-1 * sqrt(log2(e)/2), packed
//   30    log2(pi) - log2 det Lxx - (3/2) log2(2 pi)      (-inf for an unusable component)
//   31    -log2 det L' - log2(2 pi)
constexpr float kCutSq = (3.14159265358979323846f * (1.0f - 1e-6f)) * (3.14159265358979323846f * (1.0f - 1e-6f));
constexpr float kPiSq = 3.14159265358979323846f * 3.14159265358979323846f;

// ---------------------------------------------------------------------------------
// per-lane pieces
// ---------------------------------------------------------------------------------

// FP32 exp map w = R^T (nu sinc r, cos r) with the hardware sine / cosine (which take
// revolutions), square root and reciprocal
__device__ __forceinline__ void exp_map_hw(const float* R, float n0, float n1, float w[3])
{
    const float r2 = fmaf(n0, n0, n1 * n1);
    const float r = __builtin_amdgcn_sqrtf(r2);
    const float rev = r * 0.15915494309189535f;
    const float sr = __builtin_amdgcn_sinf(rev), cr = __builtin_amdgcn_cosf(rev);
    const float sc = r > 1e-4f ? sr * __builtin_amdgcn_rcpf(r) : 1.0f - r2 * (1.0f / 6.0f);
    const float v0 = n0 * sc, v1 = n1 * sc;
    for (int j = 0; j < 3; ++j) w[j] = fmaf(R[j], v0, fmaf(R[3 + j], v1, R[6 + j] * cr));
}

// The tangent candidate of one draw from a Gaussian on the tangent plane of frame R with
// factor L = (l0; l1 l2) and mean m: Box-Muller with the hardware log2 / sqrt /
// sin / cos (the sine and cosine take revolutions: sin(2 pi u2)), nu = m + L z, the exp
// map. Returns whether |nu| < pi (a draw at or beyond the cut locus is discarded).
__device__ __forceinline__ int draw_candidate(const float* R, float l0, float l1, float l2, float m0, float m1,
                                              float u1, float u2, float w[3])
{
    const float rad = __builtin_amdgcn_sqrtf(-2.0f * 0.69314718056f * __builtin_amdgcn_logf(1.0f - u1));
    const float sn = __builtin_amdgcn_sinf(u2), cs = __builtin_amdgcn_cosf(u2);
    const float z0 = rad * cs, z1 = rad * sn;
    const float n0 = fmaf(l0, z0, m0);
    const float n1 = fmaf(l1, z0, fmaf(l2, z1, m1));
    exp_map_hw(R, n0, n1, w);
    return fmaf(n0, n0, n1 * n1) < kPiSq;
}

// conditional log2-weight and mean of component T at position x
__device__ __forceinline__ float cond_component(const float* T, float x0, float x1, float x2, float& m0, float& m1)
{
    const float d0 = x0 - T[9], d1 = x1 - T[10], d2 = x2 - T[11];
    const float u0 = T[12] * d0;
    const float u1 = fmaf(T[13], d0, T[14] * d1);
    const float u2 = fmaf(T[15], d0, fmaf(T[16], d1, T[17] * d2));
    const float q = fmaf(u0, u0, fmaf(u1, u1, u2 * u2));
    m0 = fmaf(T[18], d0, fmaf(T[19], d1, T[20] * d2));
    m1 = fmaf(T[21], d0, fmaf(T[22], d1, T[23] * d2));
    return T[30] - q;
}

// Philox4x32-10 (Salmon et al. 2011)
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ void draw_uniforms(const float* uniforms, int64_t n_draws, int64_t d, uint64_t seed,
                                              float& u0, float& u1, float& u2)
{
    if (uniforms) {
        u0 = uniforms[d];
        u1 = uniforms[n_draws + d];
        u2 = uniforms[2 * n_draws + d];
    } else {
        const uint4 r = philox4x32_10(make_uint4((uint32_t)d, (uint32_t)((uint64_t)d >> 32), 0u, 0u),
                                      (uint32_t)seed, (uint32_t)(seed >> 32));
        u0 = (float)(r.x >> 8) * 0x1.0p-24f;
        u1 = (float)(r.y >> 8) * 0x1.0p-24f;
        u2 = (float)(r.z >> 8) * 0x1.0p-24f;
    }
}

// inclusive prefix sum over the G lanes of a group (lane order = component order):
// DPP row shifts inside a row of 16 lanes, shuffles across rows
template <int G>
__device__ __forceinline__ float group_inclusive_scan(float v)
{
    const int comp = (threadIdx.x & 63) % G;
    // row_shr with bound_ctrl reads 0 past the start of a 16-lane row, so a group that spans
    // whole rows needs no select; a smaller group masks its row neighbours' lanes
#define SDMM_SCAN_STEP(o)                                                                          \
    if constexpr (G > o) {                                                                         \
        const float t = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 + o, \
                                                                   0xF, 0xF, true));               \
        if constexpr (G >= 16) v += t;                                                             \
        else v += comp >= o ? t : 0.0f;                                                            \
    }
    SDMM_SCAN_STEP(1)
    SDMM_SCAN_STEP(2)
    SDMM_SCAN_STEP(4)
    SDMM_SCAN_STEP(8)
#undef SDMM_SCAN_STEP
    if constexpr (G > 16) {  // add the totals of the group's earlier rows
        const int base = (threadIdx.x & 63) - comp, row = comp >> 4;
        const float t0 = __shfl(v, base + 15);
        float add = row >= 1 ? t0 : 0.0f;
        if constexpr (G > 32) {
            const float t1 = __shfl(v, base + 31), t2 = __shfl(v, base + 47);
            add = row >= 2 ? (row >= 3 ? (t0 + t1) + t2 : t0 + t1) : add;
        }
        v += add;
    }
    return v;
}

// Sums of four values over a row of 16 lanes at once: lane i ends with the sum over the
// row of value (i & 3). Two exchange steps inside each quad leave lane i with the quad's
// sum of value (i & 3); two rotations by 4 and 8 lanes then add the four quads. The sums
// associate differently from group_sum (a different FP32 rounding, same value).
__device__ __forceinline__ float group_sum4_row16(const float (&c)[4])
{
    const int lane = threadIdx.x & 63;
    const bool b1 = (lane & 2) != 0, b0 = (lane & 1) != 0;
    // partner lane ^ 2: keep values {0,1} (bit 1 clear) or {2,3}, send the other pair
    const float k0 = b1 ? c[2] : c[0], k1 = b1 ? c[3] : c[1];
    const float s0 = b1 ? c[0] : c[2], s1 = b1 ? c[1] : c[3];
    const float a0 = k0 + dpp_f32<kDppXor2>(s0), a1 = k1 + dpp_f32<kDppXor2>(s1);
    // partner lane ^ 1: keep value (lane & 3), send the other
    const float k = b0 ? a1 : a0, sn = b0 ? a0 : a1;
    float v = k + dpp_f32<kDppXor1>(sn);
    v += dpp_f32<0x124>(v);  // row_ror:4
    v += dpp_f32<0x128>(v);  // row_ror:8
    return v;
}

// the conditioned weight pi'_k of the lane's component from the log2 weights lw of the
// group (-inf for none): exp2(lw) normalised over the group. Only a group whose sum leaves
// [2^-100, 2^100] (positions far from every component, extreme covariances, or no usable
// component) takes the maximum first (the textbook log-sum-exp); the others keep their
// values.
template <int G>
__device__ __forceinline__ float cond_weight(float lw)
{
    float e = __builtin_amdgcn_exp2f(lw);
    float den = group_sum<G>(e);
    const bool out = !(den >= 0x1p-100f && den <= 0x1p100f);
    if (__ballot(out)) {
        const float lmax = group_max<G>(lw);
        const float e2 = lmax == -INFINITY ? 0.0f : __builtin_amdgcn_exp2f(lw - lmax);
        const float den2 = group_sum<G>(e2);
        e = out ? e2 : e;
        den = out ? den2 : den;
    }
    return den > 0.0f ? e * __builtin_amdgcn_rcpf(den) : 0.0f;
}

// the log2 of the normalised weight of the lane from the log2 weights lw of the group
// (-inf for none; the result is -inf for a weight of zero), and the weight itself, by the
// same guarded normalisation as cond_weight
template <int G>
__device__ __forceinline__ float cond_log_weight(float lw, float& w)
{
    float e = __builtin_amdgcn_exp2f(lw);
    float den = group_sum<G>(e);
    float l = lw;
    const bool out = !(den >= 0x1p-100f && den <= 0x1p100f);
    if (__ballot(out)) {
        const float lmax = group_max<G>(lw);
        const float e2 = lmax == -INFINITY ? 0.0f : __builtin_amdgcn_exp2f(lw - lmax);
        const float den2 = group_sum<G>(e2);
        e = out ? e2 : e;
        den = out ? den2 : den;
        l = out ? lw - lmax : lw;
    }
    w = den > 0.0f ? e * __builtin_amdgcn_rcpf(den) : 0.0f;
    return (e > 0.0f && den > 0.0f) ? l - __builtin_amdgcn_logf(den) : -INFINITY;
}

// first chunk of component comp (clamped to K - 1) of cell qc (cell 0 when unusable)
__device__ __forceinline__ const float* table_row(const float* table, int qc, int K, int comp, bool usable)
{
    const int kk = comp < K ? comp : K - 1;
    return table + (int64_t)(usable ? qc : 0) * K * kCond + (int64_t)kk * 4;
}

// the kCond floats of one component, chunk q at q * K chunks from the first
__device__ __forceinline__ void load_row(const float* src, int K, float* T)
{
    const float4* p = reinterpret_cast<const float4*>(src);
#pragma unroll
    for (int q = 0; q < kCond / 4; ++q) {
        const float4 v = p[(int64_t)q * K];
        T[4 * q] = v.x;
        T[4 * q + 1] = v.y;
        T[4 * q + 2] = v.z;
        T[4 * q + 3] = v.w;
    }
}

// grid for a wave-strided loop over `items` work units of S per wave, in work groups of
// wpb waves
inline unsigned grid_for(int64_t items, int S, int wpb = 4)
{
    const int64_t waves = (items + S - 1) / S;
    int64_t blocks = (waves + wpb - 1) / wpb;
    const int64_t cap = 256 * 128 / wpb;  // 256 CUs x 128 waves
    if (blocks > cap) blocks = cap;
    return (unsigned)(blocks < 1 ? 1 : blocks);
}

#define SDMM_DISPATCH_G(G, CALL)         \
    switch (G) {                         \
        case 4: { constexpr int g = 4; CALL; } break;   \
        case 8: { constexpr int g = 8; CALL; } break;   \
        case 16: { constexpr int g = 16; CALL; } break; \
        case 32: { constexpr int g = 32; CALL; } break; \
        default: { constexpr int g = 64; CALL; } break; \
    }

}  // namespace sdmm
