// device_math.hpp -- gfx950 device helpers for the SDMM kernels: wave-row reductions
// with DPP, the FP32 tangent log/exp maps used in the hot loops, and the FP64 linear
// algebra of the M-step (frame, exp map, first-order transfer Jacobian, Cholesky).
//
// Paper references (Dodik et al., arXiv 2111.13094): Sec. 3.1 log-map and exp-map
// equations; Sec. 3.4 first-order covariance transfer; Appendix A Jacobians (with the
// printed typos corrected: off-diagonals nu_x nu_y c, entry (2,2) sinc + nu_y^2 c).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sdmm {

constexpr float kPiF = 3.14159265358979323846f;
constexpr double kPi = 3.14159265358979323846;
constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2Pi = 1.8378770664093453;  // log(2 pi)
constexpr int kStats = 21;                     // S0, S1[5], S2[15] (packed)
constexpr int kMirror = 48;                    // floats per component, E-step mirror
constexpr int kCond = 32;                      // floats per component, conditioning table
constexpr int kMaxK = 64;

// status bits (values are part of the C ABI)
constexpr int kSkippedFew = 1, kSkippedZeroW = 2, kBadInput = 4, kDeadComponent = 8,
              kCholFailKeptPrev = 16, kBadParams = 32;
constexpr int kFlagBadRange = 1 << 16;  // workspace-only cell flag: invalid offsets

__host__ __device__ constexpr int tri(int d, int e) { return d * (d + 1) / 2 + e; }

// Samples per work item for a cell of n samples: the configured chunk, grown for huge
// cells so that no cell has more than kMaxChunksPerCell work items (bounds the M-step's
// reduction over partials). Host and device use this same function.
constexpr int64_t kMaxChunksPerCell = 1024;
__host__ __device__ inline int64_t chunk_size_for(int64_t n, int64_t chunk)
{
    if (n <= chunk * kMaxChunksPerCell) return chunk;
    int64_t c = (n + kMaxChunksPerCell - 1) / kMaxChunksPerCell;
    return (c + 63) / 64 * 64;
}
// A cell's sample range [c0, c1) from the offsets; a range that is decreasing, negative
// or beyond n_samples is replaced by an empty one and reported as invalid.
__host__ __device__ inline bool cell_range(const int64_t* off, int c, int64_t n_samples, int64_t& c0, int64_t& c1)
{
    c0 = off[c];
    c1 = off[c + 1];
    const bool ok = c0 >= 0 && c1 >= c0 && c1 <= n_samples;
    if (!ok) c0 = c1 = 0;
    return ok;
}

__host__ __device__ inline int64_t chunks_for(int64_t n, int64_t chunk)
{
    if (n <= 0) return 1;  // empty cells still get one work item so the gate runs
    int64_t cs = chunk_size_for(n, chunk);
    return (n + cs - 1) / cs;
}

// ---------------------------------------------------------------------------------
// Row (16-lane) all-reductions with DPP. Every combination step pairs two lanes
// symmetrically, so all lanes of a group end with bitwise the same result.
// ---------------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // row_half_mirror
constexpr int kDppMirror = 0x140;     // row_mirror

// Maximum over the group, taken on an integer key that orders floats totally
// (sign-magnitude to two's complement), so each step is one fused v_max_i32 with DPP.
template <int CTRL>
__device__ __forceinline__ int dpp_max_i32(int k)
{
    return max(k, __builtin_amdgcn_update_dpp(0, k, CTRL, 0xF, 0xF, true));
}

template <int G>
__device__ __forceinline__ float group_max(float v)
{
    const int iv = __float_as_int(v);
    int k = iv ^ ((iv >> 31) & 0x7fffffff);
    if constexpr (G >= 2) k = dpp_max_i32<kDppXor1>(k);
    if constexpr (G >= 4) k = dpp_max_i32<kDppXor2>(k);
    if constexpr (G >= 8) k = dpp_max_i32<kDppHalfMirror>(k);
    if constexpr (G >= 16) k = dpp_max_i32<kDppMirror>(k);
    if constexpr (G >= 32) k = max(k, __shfl_xor(k, 16));
    if constexpr (G >= 64) k = max(k, __shfl_xor(k, 32));
    return __int_as_float(k ^ ((k >> 31) & 0x7fffffff));
}

template <int G>
__device__ __forceinline__ float group_sum(float v)
{
    if constexpr (G >= 2) v = v + dpp_f32<kDppXor1>(v);
    if constexpr (G >= 4) v = v + dpp_f32<kDppXor2>(v);
    if constexpr (G >= 8) v = v + dpp_f32<kDppHalfMirror>(v);
    if constexpr (G >= 16) v = v + dpp_f32<kDppMirror>(v);
    if constexpr (G >= 32) v = v + __shfl_xor(v, 16);
    if constexpr (G >= 64) v = v + __shfl_xor(v, 32);
    return v;
}

// ---------------------------------------------------------------------------------
// FP32 tangent log map. With w' = R w, theta = angle(w', e_z), s = |w'_xy| = sin theta:
// nu = (theta / s) w'_xy. theta / s as a function of z = cos theta is smooth on [0, 1];
// g(z) below is a degree-9 fit (max relative error 1.8e-7 in FP32 Horner form,
// generated by gen_logmap_poly.py). For z < 0, theta = pi - theta(|z|), so
// theta / s = pi / s - g(|z|). A 1e-18 offset on w'_x (below the rounding of any x
// that is not itself below 1e-11) keeps s > 0, so the exact antipode maps to (pi, 0).
// ---------------------------------------------------------------------------------
__device__ __forceinline__ float theta_over_sin_pos(float z)
{
    float p = -1.048102602e-02f;
    p = fmaf(p, z, 6.458827853e-02f);
    p = fmaf(p, z, -1.854392439e-01f);
    p = fmaf(p, z, 3.409982324e-01f);
    p = fmaf(p, z, -4.757513404e-01f);
    p = fmaf(p, z, 5.744850039e-01f);
    p = fmaf(p, z, -6.644107103e-01f);
    p = fmaf(p, z, 7.852075100e-01f);
    p = fmaf(p, z, -9.999929667e-01f);
    p = fmaf(p, z, 1.570796251e+00f);
    return p;
}

// returns f = theta / sin(theta) (= 1 / sinc |nu|) and writes nu
__device__ __forceinline__ float log_map_f32(float x, float y, float z, float& n0, float& n1)
{
    x += 1e-18f;
    const float g = theta_over_sin_pos(fabsf(z));
    const float s2 = fmaf(x, x, y * y);
    const float rs = __builtin_amdgcn_rsqf(s2);
    const float f = z < 0.0f ? fmaf(kPiF, rs, -g) : g;
    n0 = f * x;
    n1 = f * y;
    return f;
}

// FP32 exp map: w = R^T (nu sinc r, cos r), R rows (t1, t2, mu)
__device__ __forceinline__ void exp_map_f32(const float* R, float n0, float n1, float w[3])
{
    const float r = sqrtf(fmaf(n0, n0, n1 * n1));
    float sr, cr;
    __sincosf(r, &sr, &cr);
    const float sc = r > 1e-4f ? sr / r : 1.0f - r * r * (1.0f / 6.0f);
    const float v0 = n0 * sc, v1 = n1 * sc;
    for (int j = 0; j < 3; ++j) w[j] = fmaf(R[j], v0, fmaf(R[3 + j], v1, R[6 + j] * cr));
}

// ---------------------------------------------------------------------------------
// FP64 helpers for the M-step and table preparation
// ---------------------------------------------------------------------------------

// rows (t1, t2, mu): branchless orthonormal basis of Duff et al. 2017
__device__ __forceinline__ void frame64(const double mu[3], double R[9])
{
    const double sg = copysign(1.0, mu[2]);
    const double a = -1.0 / (sg + mu[2]);
    const double b = mu[0] * mu[1] * a;
    R[0] = 1.0 + sg * mu[0] * mu[0] * a;
    R[1] = sg * b;
    R[2] = -sg * mu[0];
    R[3] = b;
    R[4] = sg + mu[1] * mu[1] * a;
    R[5] = -mu[1];
    R[6] = mu[0];
    R[7] = mu[1];
    R[8] = mu[2];
}

__device__ __forceinline__ void exp_map64(const double R[9], double n0, double n1, double w[3])
{
    const double r = sqrt(n0 * n0 + n1 * n1);
    double sr, cr;
    sincos(r, &sr, &cr);
    const double sc = r > 0.0 ? sr / r : 1.0;
    const double v0 = n0 * sc, v1 = n1 * sc;
    for (int j = 0; j < 3; ++j) w[j] = R[j] * v0 + R[3 + j] * v1 + R[6 + j] * cr;
}

// (cos r - sinc r) / r^2 with its Taylor series near 0
__device__ __forceinline__ double exp_jac_c64(double r)
{
    if (r < 1e-2) {
        const double r2 = r * r;
        return -1.0 / 3.0 + r2 / 30.0 - r2 * r2 / 840.0;
    }
    double sr, cr;
    sincos(r, &sr, &cr);
    return (cr - sr / r) / (r * r);
}

// J = d(log_{mu_new} o exp_mu)/d nu at nu = m: rows(t1,t2 of R_new) * R_old^T * M(m),
// M(m) = d(nu sinc|nu|, cos|nu|)/d nu (3x2).
__device__ __forceinline__ void transfer_jac64(const double Ro[9], const double Rn[9], double m0,
                                               double m1, double J[4])
{
    const double r = sqrt(m0 * m0 + m1 * m1);
    const double s = r > 0.0 ? sin(r) / r : 1.0;
    const double c = exp_jac_c64(r);
    const double M[6] = {s + m0 * m0 * c, m0 * m1 * c, m0 * m1 * c, s + m1 * m1 * c, -m0 * s, -m1 * s};
    double RtM[6];
    for (int j = 0; j < 3; ++j)
        for (int b = 0; b < 2; ++b)
            RtM[2 * j + b] = Ro[j] * M[b] + Ro[3 + j] * M[2 + b] + Ro[6 + j] * M[4 + b];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            J[2 * a + b] = Rn[3 * a] * RtM[b] + Rn[3 * a + 1] * RtM[2 + b] + Rn[3 * a + 2] * RtM[4 + b];
}

// packed lower Cholesky of an n x n SPD matrix (n <= 5); false if not SPD
template <int n>
__device__ __forceinline__ bool chol64(const double* A, double* L)
{
#pragma unroll
    for (int d = 0; d < n; ++d) {
#pragma unroll
        for (int e = 0; e <= d; ++e) {
            double s = A[tri(d, e)];
#pragma unroll
            for (int f = 0; f < e; ++f) s -= L[tri(d, f)] * L[tri(e, f)];
            if (d == e) {
                if (!(s > 0.0) || !isfinite(s)) return false;
                L[tri(d, d)] = sqrt(s);
            } else {
                L[tri(d, e)] = s / L[tri(e, e)];
            }
        }
    }
    return true;
}

// inverse of a packed lower-triangular matrix (packed lower result)
template <int n>
__device__ __forceinline__ void tri_inv64(const double* L, double* Li)
{
#pragma unroll
    for (int d = 0; d < n; ++d) {
        Li[tri(d, d)] = 1.0 / L[tri(d, d)];
#pragma unroll
        for (int e = 0; e < d; ++e) {
            double s = 0.0;
#pragma unroll
            for (int f = e; f < d; ++f) s += L[tri(d, f)] * Li[tri(f, e)];
            Li[tri(d, e)] = -s / L[tri(d, d)];
        }
    }
}

}  // namespace sdmm
