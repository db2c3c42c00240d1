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
constexpr int kMirror = 64;                    // floats per component, E-step mirror
constexpr int kCond = 32;                      // floats per component, conditioning table
constexpr int kMaxK = 64;

// status bits (values are part of the C ABI)
constexpr int kSkippedFew = 1, kSkippedZeroW = 2, kBadInput = 4, kDeadComponent = 8,
              kCholFailKeptPrev = 16, kBadParams = 32;
constexpr int kFlagBadRange = 1 << 16;  // workspace-only cell flag: invalid offsets
constexpr int kFlagStepped = 1 << 17;   // workspace-only cell flag: the cell's M-step ran this iteration

__host__ __device__ constexpr int tri(int d, int e) { return d * (d + 1) / 2 + e; }

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

// FP64 sum over the whole wave: DPP butterflies inside each row of 16 lanes, then the
// gfx950 row swaps (permlane16 / permlane32), which hand each lane the value of lane
// l ^ 16 (l ^ 32) next to its own in a fixed order, so every lane ends with bitwise the
// same sum.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <bool ROW32>
__device__ __forceinline__ double sum_row_pair_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
    auto a = ROW32 ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false)
                   : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    auto c = ROW32 ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false)
                   : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const double d0 = __longlong_as_double(((long long)c[0] << 32) | a[0]);
    const double d1 = __longlong_as_double(((long long)c[1] << 32) | a[1]);
    return d0 + d1;
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
    v += dpp_f64<kDppXor1>(v);
    v += dpp_f64<kDppXor2>(v);
    v += dpp_f64<kDppHalfMirror>(v);
    v += dpp_f64<kDppMirror>(v);
    v = sum_row_pair_f64<false>(v);
    return sum_row_pair_f64<true>(v);
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

// returns f = theta / sin(theta) (= 1 / sinc |nu|) and writes nu; x must already carry
// the 1e-18 offset
__device__ __forceinline__ float log_map_f32_offset(float x, float y, float z, float& n0, float& n1)
{
    const float g = theta_over_sin_pos(fabsf(z));
    const float s2 = fmaf(x, x, y * y);
    const float rs = __builtin_amdgcn_rsqf(s2);
    const float f = z < 0.0f ? fmaf(kPiF, rs, -g) : g;
    n0 = f * x;
    n1 = f * y;
    return f;
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

// the radius of a tangent offset nu and its sine, cosine and sinc, evaluated once for the
// exp map and the transfer Jacobian at the same offset
struct TangentRadius64 {
    double r, sr, cr, sc;
};

__device__ __forceinline__ TangentRadius64 tangent_radius64(double n0, double n1)
{
    TangentRadius64 t;
    t.r = sqrt(n0 * n0 + n1 * n1);
    sincos(t.r, &t.sr, &t.cr);
    t.sc = t.r > 0.0 ? t.sr / t.r : 1.0;
    return t;
}

__device__ __forceinline__ void exp_map64(const double R[9], double n0, double n1, const TangentRadius64& t,
                                          double w[3])
{
    const double v0 = n0 * t.sc, v1 = n1 * t.sc;
    for (int j = 0; j < 3; ++j) w[j] = R[j] * v0 + R[3 + j] * v1 + R[6 + j] * t.cr;
}

// (cos r - sinc r) / r^2 with its Taylor series near 0
__device__ __forceinline__ double exp_jac_c64(const TangentRadius64& t)
{
    if (t.r < 1e-2) {
        const double r2 = t.r * t.r;
        return -1.0 / 3.0 + r2 / 30.0 - r2 * r2 / 840.0;
    }
    return (t.cr - t.sc) / (t.r * t.r);
}

// J = d(log_{mu_new} o exp_mu)/d nu at nu = m: rows(t1,t2 of R_new) * R_old^T * M(m),
// M(m) = d(nu sinc|nu|, cos|nu|)/d nu (3x2).
__device__ __forceinline__ void transfer_jac64(const double Ro[9], const double Rn[9], double m0, double m1,
                                               const TangentRadius64& t, double J[4])
{
    const double s = t.sc;
    const double c = exp_jac_c64(t);
    const double M[6] = {s + m0 * m0 * c, m0 * m1 * c, m0 * m1 * c, s + m1 * m1 * c, -m0 * s, -m1 * s};
    double RtM[6];
    for (int j = 0; j < 3; ++j)
        for (int b = 0; b < 2; ++b)
            RtM[2 * j + b] = Ro[j] * M[b] + Ro[3 + j] * M[2 + b] + Ro[6 + j] * M[4 + b];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            J[2 * a + b] = Rn[3 * a] * RtM[b] + Rn[3 * a + 1] * RtM[2 + b] + Rn[3 * a + 2] * RtM[4 + b];
}

// log det L of a packed 5 x 5 factor: one log of the product of the pivots, or the sum of
// their logs where that product would leave the normal FP64 range
__device__ __forceinline__ double log_det5(const double* L)
{
    const double p = L[0] * L[2] * L[5] * L[9] * L[14];
    if (p > 0x1p-1000 && p < 0x1p1000) return log(p);
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 5; ++d) s += log(L[tri(d, d)]);
    return s;
}

// packed lower Cholesky of an n x n SPD matrix (n <= 5); false if not SPD. One division
// per pivot; the off-diagonal entries multiply by the pivot's reciprocal.
template <int n>
__device__ __forceinline__ bool chol64(const double* A, double* L, double* inv_out = nullptr)
{
    double inv[n];
#pragma unroll
    for (int d = 0; d < n; ++d) {
#pragma unroll
        for (int e = 0; e <= d; ++e) {
            double s = A[tri(d, e)];
#pragma unroll
            for (int f = 0; f < e; ++f) s -= L[tri(d, f)] * L[tri(e, f)];
            if (d == e) {
                if (!(s > 0.0) || !isfinite(s)) return false;
                const double r = sqrt(s);
                L[tri(d, d)] = r;
                inv[d] = 1.0 / r;
                if (inv_out) inv_out[d] = inv[d];
            } else {
                L[tri(d, e)] = s * inv[e];
            }
        }
    }
    return true;
}

// inverse of a packed lower-triangular matrix (packed lower result)
// inverse of a packed lower-triangular factor; the reciprocals of its diagonal may come in
// from the factorisation that formed it (inv_diag)
template <int n>
__device__ __forceinline__ void tri_inv64(const double* L, double* Li, const double* inv_diag = nullptr)
{
#pragma unroll
    for (int d = 0; d < n; ++d) {
        Li[tri(d, d)] = inv_diag ? inv_diag[d] : 1.0 / L[tri(d, d)];
#pragma unroll
        for (int e = 0; e < d; ++e) {
            double s = 0.0;
#pragma unroll
            for (int f = e; f < d; ++f) s += L[tri(d, f)] * Li[tri(f, e)];
            Li[tri(d, e)] = -s * Li[tri(d, d)];
        }
    }
}

// The EM part of a component's FP32 E-step mirror (floats 0-27: frame R, mu_x, the
// inverse factor scaled by sqrt(log2(e) / 2), and c2 = (log pi - log det L -
// (5/2) log 2 pi) log2(e), also returned in FP64) from its weight, frame, positional mean
// and packed covariance factor L with the reciprocals Ld of its diagonal; Li receives
// L^-1 (unscaled).
__device__ __forceinline__ void mirror_core(double pi, const double* R, const double* mux, const double* L,
                                            const double* Ld, float* out, double& c2, double* Li)
{
    tri_inv64<5>(L, Li, Ld);
    const double logdet = log_det5(L);
    const double scale = sqrt(0.5 * kLog2e);
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i] = (float)R[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) out[9 + d] = (float)mux[d];
#pragma unroll
    for (int i = 0; i < 15; ++i) out[12 + i] = (float)(Li[i] * scale);
    c2 = (log(pi) - logdet - 2.5 * kLn2Pi) * kLog2e;
    out[27] = (float)c2;
}

}  // namespace sdmm
