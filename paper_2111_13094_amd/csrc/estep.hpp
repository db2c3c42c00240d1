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

#include <type_traits>

#include "device_math.hpp"

namespace sdmm {

enum { kAccTwoSum = 0, kAccPlain = 1, kAccFp64 = 2 };
constexpr int kFoldEvery = 64;  // steps between folds of the FP32 block sums

// running sums: FP32 block sums over kFoldEvery steps (a lane's samples of a work item of
// up to 256 samples fit one block), folded by TwoSum into an FP32 running total whose
// rounding error opens the next block (compensated), kept as one plain FP32 sum, or
// folded into FP64 (precision variants)
template <int ACC>
struct RunSum;

template <>
struct RunSum<kAccTwoSum> {
    float blk = 0.0f, hi = 0.0f;
    __device__ __forceinline__ void add(float v) { blk += v; }
    __device__ __forceinline__ void fma_add(float a, float b) { blk = fmaf(a, b, blk); }
    // hi + blk = s + err exactly (Knuth's TwoSum); s becomes the total and err the start
    // of the next block, so hi + blk always equals the folded sum exactly
    __device__ __forceinline__ void fold()
    {
        const float s = hi + blk;
        const float bb = s - hi;
        blk = (hi - (s - bb)) + (blk - bb);
        hi = s;
    }
    __device__ __forceinline__ double total() { return (double)hi + (double)blk; }
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
    __device__ __forceinline__ double total() { return hi + (double)blk; }
};

// statistics per component and the per-item record layout: statistic s of component k
// at s * G + k (G = K rounded up to a power of two, at least 4), then the per-item extras
template <bool ADJ>
struct ChunkLayout {
    static constexpr int kNStat = ADJ ? 23 : 21;       // S0, S1[5], S2[15] (+ g_delta[2])
    static constexpr int kNRed = kNStat + (ADJ ? 4 : 3); // + W, M, negatives (+ LL)
    static __host__ __device__ constexpr int record(int G) { return (kNStat * G + (kNRed - kNStat) + 1) & ~1; }
};

// Element type of the per-item records: FP32 for the EM passes with FP32 block sums (the
// item's FP64 total is rounded once; a record's rounding, 2^-24 relative, stays below
// the FP32 accumulation error within the item), FP64 for the FP64-sum and adjoint passes.
template <int ACC, bool ADJ>
using RecordT = typename std::conditional<(ACC == kAccFp64 || ADJ), double, float>::type;

// Sums the records of one cell's items 0, 2^stride_log2, 2 * 2^stride_log2, ... below
// n_items (record slots from `first`) in item order, one column per lane (all 64 lanes
// of the wave, which must be uniform in first/n_items), with the loads of several records
// in flight: column q * 64 + lane of the record (statistic s of component k at s * G + k,
// then the extras) ends in v[q]. With stride 2^(4 L) the summed records are the level-L
// leaders of the record tree (see tree_kernel). RB0 records per round trip by default
// (fewer when a record spans many registers).
template <int G, int NS, int NX, int RB0 = 4, typename RT = double>
__device__ __forceinline__ void sum_cell_columns(const RT* __restrict__ records, int64_t first, int64_t n_items,
                                                 int PS, int stride_log2, double (&v)[(NS * G + NX + 63) / 64])
{
    constexpr int NCOL = NS * G + NX, NQ = (NCOL + 63) / 64;
    const int lane = threadIdx.x & 63;
    const int64_t n = (n_items + (int64_t(1) << stride_log2) - 1) >> stride_log2;  // records to sum
    const int64_t step = (int64_t)PS << stride_log2;                                 // elements between them
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = 0.0;
    // RB records per round trip (twice as many for FP32 records, held as loaded). Every
    // load is issued, at an index clamped to the cell's last record and the record's last
    // column (no branch, one wait per round trip); what lies past them adds an exact zero,
    // so the sum is the same as record by record
    constexpr int RB = (NQ > 6 ? 2 : RB0) * (sizeof(RT) == 4 ? 2 : 1);
    for (int64_t j = 0; j < n; j += RB) {
        const RT* r0 = records + first * PS + j * step;
        RT a[RB][NQ];
#pragma unroll
        for (int u = 0; u < RB; ++u)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int64_t uu = min(j + u, n - 1) - j;
                a[u][q] = r0[uu * step + min(q * 64 + lane, NCOL - 1)];
            }
#pragma unroll
        for (int u = 0; u < RB; ++u)
#pragma unroll
            for (int q = 0; q < NQ; ++q) v[q] += (j + u < n && q * 64 + lane < NCOL) ? (double)a[u][q] : 0.0;
    }
}

// The same sums handed to lane k < G as its component's statistics S[s] = column
// s * G + k, and to every lane as the extras X[i] = column NS * G + i.
template <int G, int NS, int NX, typename RT>
__device__ __forceinline__ void sum_cell_records(const RT* __restrict__ records, int64_t first, int64_t n_items,
                                                 int PS, int stride_log2, double (&S)[NS], double (&X)[NX])
{
    constexpr int NQ = (NS * G + NX + 63) / 64;
    double v[NQ];
    sum_cell_columns<G, NS, NX>(records, first, n_items, PS, stride_log2, v);
    const int k = (threadIdx.x & 63) % G;
#pragma unroll
    for (int s = 0; s < NS; ++s) S[s] = __shfl(v[(s * G) / 64], (s * G) % 64 + k);
#pragma unroll
    for (int i = 0; i < NX; ++i) X[i] = __shfl(v[(NS * G + i) / 64], (NS * G + i) % 64);
}

// Mirror slots: 0-8 R, 9-11 mu_x, 12-26 scaled Linv, 27 shifted log2 constant, 28-29 twist
// rates, 30 the cell's log2 shift, 31 unused, 32-40 R residue, 41-43 mu_x residue,
// 44-58 scaled Linv residue, 59 residue of the shifted log2 constant, 60-61 twist rate
// residues, 62-63 unused.
constexpr int kMirShift = 30;
constexpr int kMirrorLite = 32;  // floats of a mirror that the EM passes read

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
// c * log2(e) with c = log pi - log det L - (5/2) log 2 pi (1, returned in c2 and shifted
// per cell by set_mirror_shift), and with FULL the frame twist rates (2) used by the
// adjoint and the FP32 rounding residues of R, mu_x, the scaled Linv and the shifted
// constant. With them the adjoint pass forms tangent coordinates to FP32 relative accuracy
// and the quadratic form in FP64 (its gradients are small differences near stationarity,
// and for strongly correlated components the quadratic form cancels). The EM passes read
// only the first kMirrorLite floats, which is all a lite mirror (FULL false) writes.
// ---------------------------------------------------------------------------------

// The mirror of a component from its weight, frame R (rows t1, t2, mu), positional mean and
// packed covariance factor L with the reciprocals Ld of its diagonal (mud, the directional
// mean, is read only with FULL, for the twist rates).
template <bool FULL>
__device__ __forceinline__ void mirror_from_factor(double pi, const double* mud, const double* R, const double* mux,
                                                   const double* L, const double* Ld, float* out, double& c2)
{
    double Li[15];
    mirror_core(pi, R, mux, L, Ld, out, c2, Li);
    if constexpr (!FULL) {
        out[28] = out[29] = out[30] = out[31] = 0.0f;
        return;
    }
    const double scale = sqrt(0.5 * kLog2e);
    double phi[2];
    frame_twist64(mud, R, phi);
    out[28] = (float)phi[0];
    out[29] = (float)phi[1];
    out[30] = out[31] = 0.0f;
    for (int i = 0; i < 9; ++i) out[32 + i] = (float)(R[i] - (double)out[i]);
    for (int d = 0; d < 3; ++d) out[41 + d] = (float)(mux[d] - (double)out[9 + d]);
    for (int i = 0; i < 15; ++i) out[44 + i] = (float)(Li[i] * scale - (double)out[12 + i]);
    out[60] = (float)(phi[0] - (double)out[28]);
    out[61] = (float)(phi[1] - (double)out[29]);
    out[62] = out[63] = 0.0f;
}

// The mirror of a component from its parameters; returns false and writes an inert mirror
// (identity frame and factor) when the component is unusable.
template <bool FULL>
__device__ inline bool write_mirror(double pi, const double* mud, const double* mux, const double* cov,
                                    float* out, double& c2)
{
    bool ok = isfinite(pi) && pi >= 0.0;
    for (int d = 0; d < 3; ++d) ok = ok && isfinite(mud[d]) && isfinite(mux[d]);
    double L[15], Ld[5];
    ok = ok && chol64<5>(cov, L, Ld);
    if (!ok) {
        for (int i = 0; i < (FULL ? kMirror : kMirrorLite); ++i) out[i] = 0.0f;
        out[0] = out[4] = out[8] = 1.0f;
        const int diag[5] = {0, 2, 5, 9, 14};
        for (int d = 0; d < 5; ++d) out[12 + diag[d]] = 1.0f;
        c2 = -INFINITY;
        return false;
    }
    double R[9];
    frame64(mud, R);
    mirror_from_factor<FULL>(pi, mud, R, mux, L, Ld, out, c2);
    return true;
}

// Shifts the log2 constants of one cell by (max over its components + 1), so that every
// log2 density the E-step forms is negative (the maximum then reduces over the float bit
// patterns as integers) and stays small where it matters (no rounding of a large common
// constant). Inert components (`usable` false: the cell is gated as BAD_PARAMS) get -1. A
// usable component of weight zero keeps the constant -inf, so its responsibility is
// exactly zero, as the E-step of Sec. 3.2 gives (r proportional to pi_k p_k). `shift` is
// the same for all lanes of the cell.
template <bool FULL>
__device__ inline void set_mirror_shift(float* out, double c2, double shift, bool usable)
{
    if (!usable || !isfinite(c2)) {
        out[27] = usable ? -INFINITY : -1.0f;
        if constexpr (FULL) out[59] = 0.0f;
    } else {
        const double v = c2 - shift;
        out[27] = (float)v;
        if constexpr (FULL) out[59] = (float)(v - (double)out[27]);
    }
    out[kMirShift] = (float)shift;
}

// stores a mirror built in registers with 16-byte stores (the lite part only unless FULL)
template <bool FULL>
__device__ __forceinline__ void store_mirror(float* __restrict__ dst, const float (&m)[kMirror])
{
    float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
    for (int q = 0; q < (FULL ? kMirror : kMirrorLite) / 4; ++q)
        d4[q] = make_float4(m[4 * q], m[4 * q + 1], m[4 * q + 2], m[4 * q + 3]);
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

__device__ __forceinline__ SampleRegs load_sample_at(const float* const* ch, uint32_t b)
{
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

// W = sum w (FP64 per lane, then a wave reduction), M = #{w > 0}, negatives = #{w < 0}
// over [s0, s1), one sample per lane of one wave; the counts come from ballots (scalar
// unit). Every lane returns the totals.
__device__ __forceinline__ void weight_pass(const float* __restrict__ wch, int64_t s0, int64_t s1, double& W,
                                            double& M, double& neg)
{
    const int lane = threadIdx.x & 63;
    double sw = 0.0;
    uint32_t cnt = 0, ng = 0;
    for (int64_t b = s0; b < s1; b += 64) {  // wave-uniform trip count
        const int64_t i = b + lane;
        const float w = i < s1 ? wch[i] : 0.0f;
        sw += (double)w;
        cnt += (uint32_t)__popcll(__ballot(w > 0.0f));
        ng += (uint32_t)__popcll(__ballot(w < 0.0f));
    }
    W = wave_sum_f64(sw);
    M = (double)cnt;
    neg = (double)ng;
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

// Maximum over the group of negative floats: for negative IEEE floats the integer order
// of the bit patterns is reversed, so the float maximum is the integer minimum, one fused
// v_min_i32 with DPP per step.
template <int CTRL>
__device__ __forceinline__ int dpp_min_i32(int k)
{
    return min(k, __builtin_amdgcn_update_dpp(0, k, CTRL, 0xF, 0xF, true));
}

template <int G>
__device__ __forceinline__ float group_max_negative(float v)
{
    int k = __float_as_int(v);
    if constexpr (G >= 2) k = dpp_min_i32<kDppXor1>(k);
    if constexpr (G >= 4) k = dpp_min_i32<kDppXor2>(k);
    if constexpr (G >= 8) k = dpp_min_i32<kDppHalfMirror>(k);
    if constexpr (G >= 16) k = dpp_min_i32<kDppMirror>(k);
    if constexpr (G >= 32) k = min(k, __shfl_xor(k, 16));
    if constexpr (G >= 64) k = min(k, __shfl_xor(k, 32));
    return __int_as_float(k);
}

// largest c in [0, C) with c + off[c] / 2^ps <= t (0 if none), by a 64-ary search of the wave
__device__ __forceinline__ int find_slot_cell(const int64_t* __restrict__ off, int C, int ps, int64_t t)
{
    const int lane = threadIdx.x & 63;
    int a = 0, n = C;
    while (n > 1) {
        const int step = (n + 63) / 64;
        const int idx = a + lane * step;
        const bool le = idx < a + n && (int64_t)idx + (off[idx] >> ps) <= t;
        const uint64_t m = __ballot(le);
        const int j = m ? 63 - __builtin_clzll(m) : 0;
        const int end = a + n;
        a += j * step;
        n = min(step, end - a);
    }
    return a;
}

// E-step work items of cell c: its samples [off[c], off[c+1]) cut from the cell's first
// sample into ceil(n / P) items of at most P = 2^ps samples (one empty item for an empty
// cell, so that every cell has a record and an M-step), item j in record slot first + j
// with first = c + off[c] / P. False for a range outside [0, N] or a decreasing one.
__device__ __forceinline__ bool cell_items(const int64_t* off, int64_t N, int c, int ps, int64_t& first,
                                           int64_t& n_items)
{
    const int64_t c0 = off[c], c1 = off[c + 1];
    if (!(c0 >= 0 && c1 >= c0 && c1 <= N)) return false;
    first = c + (c0 >> ps);
    n_items = c1 > c0 ? (c1 - c0 + (int64_t(1) << ps) - 1) >> ps : 1;
    return true;
}

// E-step of one segment [s0, s1) of a cell by one wave. mirror_cell points at the cell's
// K FP32 mirrors. Writes the segment record part[] (RecordT, from the FP64 totals) from
// lanes < G.
template <int G, int ACC, bool JAC, bool ADJ>
__device__ __forceinline__ void estep_segment(const float* __restrict__ smp, int64_t N, int64_t s0, int64_t s1,
                                              const float* __restrict__ mirror_cell, int K,
                                              RecordT<ACC, ADJ>* __restrict__ part)
{
    using CL = ChunkLayout<ADJ>;
    using RT = RecordT<ACC, ADJ>;
    constexpr int NS = CL::kNStat, NR = CL::kNRed;
    constexpr int S = 64 / G;
    const int lane = threadIdx.x & 63;
    const int comp = lane % G, slot = lane / G;
    const int kk = comp < K ? comp : K - 1;

    const float4* mp = reinterpret_cast<const float4*>(mirror_cell + (int64_t)kk * kMirror);
    float P[60];
#pragma unroll
    for (int q = 0; q < (ADJ ? 15 : 7); ++q) {
        const float4 v = mp[q];
        P[4 * q] = v.x;
        P[4 * q + 1] = v.y;
        P[4 * q + 2] = v.z;
        P[4 * q + 3] = v.w;
    }
    const float c2 = comp < K ? P[27] : -INFINITY;

    // channel bases start at the segment so that lane offsets fit in 32 bits
    const float* ch[7];
#pragma unroll
    for (int a = 0; a < 7; ++a) ch[a] = smp + (int64_t)a * N + s0;

    RunSum<ACC> acc[NS];
    RunSum<ACC> accll;

    const uint32_t n = (uint32_t)(s1 - s0);
    const uint32_t last = n > 0 ? n - 1 : 0;

    // one (sample, component) pair per lane
    auto body = [&](const SampleRegs& cur, bool valid) {
        const float w = valid ? cur.w : 0.0f;

        // tangent coordinates y = (log_mu w, p - mu_x); the 1e-18 offset on w'_x keeps
        // the antipode away from 0/0 in the log map
        float xr = fmaf(P[0], cur.ox, fmaf(P[1], cur.oy, fmaf(P[2], cur.oz, 1e-18f)));
        float yr = fmaf(P[3], cur.ox, fmaf(P[4], cur.oy, P[5] * cur.oz));
        float zr = fmaf(P[6], cur.ox, fmaf(P[7], cur.oy, P[8] * cur.oz));
        if constexpr (ADJ) {  // add the residue of the FP32-rounded frame
            xr += fmaf(P[32], cur.ox, fmaf(P[33], cur.oy, P[34] * cur.oz));
            yr += fmaf(P[35], cur.ox, fmaf(P[36], cur.oy, P[37] * cur.oz));
            zr += fmaf(P[38], cur.ox, fmaf(P[39], cur.oy, P[40] * cur.oz));
        }
        float y0, y1;
        const float f = log_map_f32_offset(xr, yr, zr, y0, y1);
        float y2 = cur.px - P[9], y3 = cur.py - P[10], y4 = cur.pz - P[11];
        if constexpr (ADJ) {
            y2 -= P[41];
            y3 -= P[42];
            y4 -= P[43];
        }

        // shifted log2 of pi_k N5(y; 0, Sigma_k) through the scaled inverse Cholesky factor
        float z0, z1, z2, z3, z4, l;
        double ld = 0.0;
        if constexpr (ADJ) {  // FP64 quadratic form from the hi/lo factor and constant
            auto Lq = [&](int q) { return (double)P[12 + q] + (double)P[44 + q]; };
            const double e0 = y0, e1 = y1, e2 = y2, e3 = y3, e4 = y4;
            const double w0 = Lq(0) * e0;
            const double w1 = fma(Lq(1), e0, Lq(2) * e1);
            const double w2 = fma(Lq(3), e0, fma(Lq(4), e1, Lq(5) * e2));
            const double w3 = fma(Lq(6), e0, fma(Lq(7), e1, fma(Lq(8), e2, Lq(9) * e3)));
            const double w4 = fma(Lq(10), e0, fma(Lq(11), e1, fma(Lq(12), e2, fma(Lq(13), e3, Lq(14) * e4))));
            const double c2d = comp < K ? (double)P[27] + (double)P[59] : -INFINITY;
            ld = c2d - w0 * w0 - w1 * w1 - w2 * w2 - w3 * w3 - w4 * w4;
            z0 = (float)w0;
            z1 = (float)w1;
            z2 = (float)w2;
            z3 = (float)w3;
            z4 = (float)w4;
            l = (float)ld;
        } else {
            z0 = P[12] * y0;
            z1 = fmaf(P[13], y0, P[14] * y1);
            z2 = fmaf(P[15], y0, fmaf(P[16], y1, P[17] * y2));
            z3 = fmaf(P[18], y0, fmaf(P[19], y1, fmaf(P[20], y2, P[21] * y3)));
            z4 = fmaf(P[22], y0, fmaf(P[23], y1, fmaf(P[24], y2, fmaf(P[25], y3, P[26] * y4))));
            l = fmaf(-z0, z0, c2);
            l = fmaf(-z1, z1, l);
            l = fmaf(-z2, z2, l);
            l = fmaf(-z3, z3, l);
            l = fmaf(-z4, z4, l);
        }
        if constexpr (JAC) l += __log2f(f);  // solid-angle density: times f (may be > 0)

        // responsibilities: log-sum-exp across the component lanes of this sample
        float lmax = 0.0f, e, den;
        if constexpr (JAC || ADJ) {
            if constexpr (JAC) lmax = group_max<G>(l);
            else lmax = group_max_negative<G>(l);
            if constexpr (ADJ) e = __builtin_amdgcn_exp2f((float)(ld - (double)lmax));
            else e = __builtin_amdgcn_exp2f(l - lmax);
            den = group_sum<G>(e);
        } else {
            // every l is at most -1 (the per-cell shift), so exp2(l) needs no maximum unless
            // the sample's whole sum is tiny; such a group (rare: far from every component)
            // takes the max-shifted form, the others keep their values
            e = __builtin_amdgcn_exp2f(l);
            den = group_sum<G>(e);
            if (__ballot(den < 0x1p-100f)) {
                const float m = group_max_negative<G>(l);
                const float e2 = __builtin_amdgcn_exp2f(l - m);
                const float den2 = group_sum<G>(e2);
                const bool redo = den < 0x1p-100f;
                e = redo ? e2 : e;
                den = redo ? den2 : den;
            }
        }
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
            // shifted log2 p(y_i) (the same value in every lane of the group); the cell's
            // shift is added back in FP64 by the gradient assembly
            accll.add(w * (lmax + __log2f(den)));
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

    // full steps (every slot valid) two at a time with alternating prefetch registers,
    // then at most two tail steps with the validity test. Inside the loop both loads of an
    // iteration are full steps, so they need no clamp and take byte offsets that advance
    // by one add each; the last pair of full steps clamps its prefetch and leaves its open
    // blocks to total().
    const uint32_t full = n / S, steps = (n + S - 1) / S;  // wave-uniform
    uint32_t i = (uint32_t)slot;
    uint32_t it = 0;
    SampleRegs a{}, b{};
    if (n > 0) a = load_sample(ch, min(i, last));
    uint32_t ob = (i + S) * 4u, oa = (i + 2 * S) * 4u;
    for (; it + 2 < full; it += 2) {
        b = load_sample_at(ch, ob);  // step it + 1
        body(a, true);
        a = load_sample_at(ch, oa);  // step it + 2 < full
        body(b, true);
        ob += 8u * S;
        oa += 8u * S;
        i += 2 * S;
        if (((it + 2) % kFoldEvery) == 0) fold_all();
    }
    if (it + 2 == full) {
        b = load_sample(ch, i + S);
        body(a, true);
        a = load_sample(ch, min(i + 2 * S, last));
        body(b, true);
        i += 2 * S;
        it += 2;
    }
    for (; it < steps; ++it) {  // at most one full and one partial step
        body(a, i <= last);
        i += S;
        a = load_sample(ch, min(i, last));
    }

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
        for (int s = 0; s < NS; ++s) part[s * G + comp] = (RT)v[s];
        if (comp == 0) {
#pragma unroll
            for (int s = NS; s < NR; ++s) part[NS * G + (s - NS)] = (RT)v[s];
        }
    }
}

// ---------------------------------------------------------------------------------
// Record tree for cells with many items. Level l >= 1 groups a cell's items in blocks of
// 16^l; the level-l leader of a block (its first item's record) receives the sum, in
// order, of the block's up to 16 level-(l-1) leaders. Level-l leaders are exactly the
// items of size P * 16^l, so a wave finds its leader by the same slot search with the
// shift ps + 4 l. Levels run while the largest cell would leave more than kTreeTop
// leaders for the M-step; the M-step then sums at most kTreeTop leader records.
// ---------------------------------------------------------------------------------
constexpr int kTreeLog2R = 4;
constexpr int kTreeTop = 128;

__host__ __device__ inline int tree_levels(int64_t max_items)
{
    int L = 0;
    while (max_items > kTreeTop) {
        max_items = (max_items + (1 << kTreeLog2R) - 1) >> kTreeLog2R;
        ++L;
    }
    return L;
}

// record-tree levels to launch for N samples in items of P when no cell holds more than
// max_cell samples (max_cell <= 0: no bound); a cell above the bound needs more levels
// than launched, and the M-step then sums the leaders of the highest launched level
inline int tree_levels_launched(int64_t N, int64_t P, int32_t max_cell)
{
    const int64_t cap = (max_cell > 0 && max_cell < N) ? max_cell : N;
    return tree_levels((cap + P - 1) / P);
}

// record-tree level whose leaders the M-step sums: the levels the largest cell needs,
// at most those launched (control words: [1] most items in a cell, [2] levels launched)
__device__ __forceinline__ int tree_levels_done(const int32_t* __restrict__ control)
{
    return min(tree_levels(control[1]), control[2]);
}

// the level-`level` leader in level slot t, if any, sums its block (see tree_kernel)
template <int G, int NS, int NX, typename RT>
__device__ __forceinline__ void tree_leader(const int64_t* __restrict__ off, int64_t N, int C, int ps, int level,
                                            int64_t t, RT* __restrict__ records, int PS)
{
    constexpr int NCOL = NS * G + NX, NQ = (NCOL + 63) / 64;
    const int psl = ps + kTreeLog2R * level;
    const int c = find_slot_cell(off, C, psl, t);
    int64_t first, n_items;
    if (!cell_items(off, N, c, ps, first, n_items)) return;
    const int64_t b = t - (c + (off[c] >> psl));
    const int64_t leaders = (n_items + (int64_t(1) << (kTreeLog2R * level)) - 1) >> (kTreeLog2R * level);
    if (b < 0 || b >= leaders) return;
    const int64_t sub = int64_t(1) << (kTreeLog2R * (level - 1));
    const int64_t base = b << (kTreeLog2R * level);
    const int64_t count = min((int64_t)(1 << kTreeLog2R), (n_items - base + sub - 1) / sub);
    if (count <= 1) return;
    const int lane = threadIdx.x & 63;
    RT* r0 = records + (first + base) * PS;
    const int64_t step = (int64_t)PS * sub;
    double v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = (q * 64 + lane < NCOL) ? (double)r0[q * 64 + lane] : 0.0;
    for (int64_t i = 1; i < count; ++i) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (q * 64 + lane < NCOL) v[q] += (double)r0[i * step + q * 64 + lane];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (q * 64 + lane < NCOL) r0[q * 64 + lane] = (RT)v[q];
}

// control[0]: offsets valid, control[1]: the largest item count of a cell (setup kernel).
// A fixed grid strides over the level slots, so a level that is not needed costs one
// small dispatch.
template <int G, int NS, int NX, typename RT>
__global__ __launch_bounds__(256) void tree_kernel(const int64_t* __restrict__ off, int64_t N, int C, int ps,
                                                   int level, int64_t slot_lo, int64_t slot_hi,
                                                   const int32_t* __restrict__ control, void* __restrict__ records_v,
                                                   int PS)
{
    if (!control[0] || level > tree_levels(control[1])) return;  // a level this batch does not need
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t t = slot_lo + wave; t < slot_hi; t += nwaves)
        tree_leader<G, NS, NX, RT>(off, N, C, ps, level, t, static_cast<RT*>(records_v), PS);
}

// ---------------------------------------------------------------------------------
// FP64 adjoint pass (verification mode): the same statistics, log-likelihood and
// directional-mean gradient terms as estep_segment<G, *, false, true>, with the frame,
// positional mean, scaled inverse factor and constant taken from their hi/lo FP32 pairs
// and every per-pair quantity (rotation, log map, quadratic form, responsibilities,
// products, sums) in FP64. Records have the adjoint layout.
// ---------------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ double group_max_f64(double v)
{
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
template <int G>
__device__ __forceinline__ double group_sum_f64(double v)
{
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o);
    return v;
}

template <int G>
__device__ void estep_segment_adj64(const float* __restrict__ smp, int64_t N, int64_t s0, int64_t s1,
                                    const float* __restrict__ mirror_cell, int K, double* __restrict__ part)
{
    using CL = ChunkLayout<true>;
    constexpr int NS = CL::kNStat, NR = CL::kNRed;
    constexpr int S = 64 / G;
    const int lane = threadIdx.x & 63;
    const int comp = lane % G, slot = lane / G;
    const int kk = comp < K ? comp : K - 1;
    const float* P = mirror_cell + (int64_t)kk * kMirror;
    double R[9], mx[3], Li[15];
    for (int i = 0; i < 9; ++i) R[i] = (double)P[i] + (double)P[32 + i];
    for (int d = 0; d < 3; ++d) mx[d] = (double)P[9 + d] + (double)P[41 + d];
    for (int q = 0; q < 15; ++q) Li[q] = (double)P[12 + q] + (double)P[44 + q];
    const double c2 = comp < K ? (double)P[27] + (double)P[59] : -INFINITY;
    const double ph0 = (double)P[28] + (double)P[60], ph1 = (double)P[29] + (double)P[61];

    double acc[NS];
    for (int q = 0; q < NS; ++q) acc[q] = 0.0;
    double accll = 0.0;
    const int64_t n = s1 - s0;
    const int64_t steps = (n + S - 1) / S;
    for (int64_t it = 0; it < steps; ++it) {
        const int64_t ii = s0 + it * S + slot;
        const bool valid = ii < s1;
        const int64_t i = valid ? ii : s1 - 1;
        const double ox = smp[i], oy = smp[N + i], oz = smp[2 * N + i];
        const double px = smp[3 * N + i], py = smp[4 * N + i], pz = smp[5 * N + i];
        const double w = valid ? (double)smp[6 * N + i] : 0.0;
        // rotation into the component frame and the log map
        const double xr = R[0] * ox + R[1] * oy + R[2] * oz;
        const double yr = R[3] * ox + R[4] * oy + R[5] * oz;
        const double zr = R[6] * ox + R[7] * oy + R[8] * oz;
        const double s2 = xr * xr + yr * yr;
        const double sn = sqrt(s2);
        double f, fp, y0, y1;
        if (sn > 0.0) {
            f = atan2(sn, zr) / sn;
            // d(theta / sin theta)/dz = (z f - 1) / s^2, with its series near z = 1
            fp = (s2 < 1e-8 && zr > 0.0) ? -zr * (1.0 / 3.0 + 0.3 * s2) : (zr * f - 1.0) / s2;
            y0 = f * xr;
            y1 = f * yr;
        } else {  // on the axis: the mean itself, or its antipode (cut locus, (pi, 0))
            f = 1.0;
            fp = -1.0 / 3.0;
            y0 = zr > 0.0 ? 0.0 : kPi;
            y1 = 0.0;
        }
        const double y[5] = {y0, y1, px - mx[0], py - mx[1], pz - mx[2]};
        double z[5];
        z[0] = Li[0] * y[0];
        z[1] = Li[1] * y[0] + Li[2] * y[1];
        z[2] = Li[3] * y[0] + Li[4] * y[1] + Li[5] * y[2];
        z[3] = Li[6] * y[0] + Li[7] * y[1] + Li[8] * y[2] + Li[9] * y[3];
        z[4] = Li[10] * y[0] + Li[11] * y[1] + Li[12] * y[2] + Li[13] * y[3] + Li[14] * y[4];
        const double l = c2 - (z[0] * z[0] + z[1] * z[1] + z[2] * z[2] + z[3] * z[3] + z[4] * z[4]);
        const double lmax = group_max_f64<G>(l);
        const double e = exp2(l - lmax);
        const double den = group_sum_f64<G>(e);
        const double wr = w * (e / den);
        acc[0] += wr;
        for (int d = 0; d < 5; ++d) acc[1 + d] += wr * y[d];
        for (int d = 0; d < 5; ++d)
            for (int b = 0; b <= d; ++b) acc[6 + tri(d, b)] += wr * y[d] * y[b];
        accll += w * (lmax + log2(den));
        // u = L^-T z on the directional coordinates (scaled like the FP32 pass)
        const double u0 = Li[0] * z[0] + Li[1] * z[1] + Li[3] * z[2] + Li[6] * z[3] + Li[10] * z[4];
        const double u1 = Li[2] * z[1] + Li[4] * z[2] + Li[7] * z[3] + Li[11] * z[4];
        const double dx0 = ph0 * yr - zr, dx1 = ph1 * yr;
        const double dy0 = -ph0 * xr, dy1 = -ph1 * xr - zr;
        const double D00 = fp * xr * xr + f * dx0, D01 = fp * yr * xr + f * dx1;
        const double D10 = fp * xr * yr + f * dy0, D11 = fp * yr * yr + f * dy1;
        acc[NS - 2] += wr * (D00 * u0 + D10 * u1);
        acc[NS - 1] += wr * (D01 * u0 + D11 * u1);
    }
    double v[NR];
    for (int q = 0; q < NS; ++q) v[q] = acc[q];
    double W, M, neg;
    weight_pass(smp + 6 * N, s0, s1, W, M, neg);
    v[NS] = slot == 0 ? W : 0.0;
    v[NS + 1] = slot == 0 ? M : 0.0;
    v[NS + 2] = slot == 0 ? neg : 0.0;
    v[NS + 3] = accll;
#pragma unroll
    for (int o = G; o < 64; o <<= 1) {
#pragma unroll
        for (int q = 0; q < NR; ++q) v[q] += __shfl_xor(v[q], o);
    }
    if (lane < G) {
        for (int q = 0; q < NS; ++q) part[q * G + comp] = v[q];
        if (comp == 0)
            for (int q = NS; q < NR; ++q) part[NS * G + (q - NS)] = v[q];
    }
}

}  // namespace sdmm
