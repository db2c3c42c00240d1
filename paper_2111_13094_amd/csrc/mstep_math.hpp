// mstep_math.hpp -- the FP64 MAP update of one mixture component from its Robbins-Monro
// blended statistics (Sec. 3.2 mean update through the exp map, Sec. 3.4 first-order
// transport of the scatter, Sec. 4.3 MAP weights and covariances), shared by the batched
// M-step and the stepwise (per-sample) kernel.
#pragma once

#include "common.hpp"

namespace sdmm {

// Robbins-Monro weight of step j: 1 for the first step, then eta or (rm_beta j + 1)^-rm_alpha
__device__ __forceinline__ double rm_eta(const DevOpts& o, int j)
{
    return j == 0 ? 1.0 : (o.eta_mode == 0 ? o.eta : pow(o.rm_beta * j + 1.0, -o.rm_alpha));
}

// Updates one component (arrays of the component: mud[3], mux[3], cov[15], s0[1],
// s2[15]; its current means mu_in, mux_in passed by value, so that the caller can load
// them early) from the blended statistics hS0, hS1, hS2 and normaliser hW with prior
// strength beta; bar0 = hS0 / hW. A dead component (bar0 at or below the threshold) keeps its
// mean and covariance and stores the blended statistics. Otherwise the mean moves by
// m = hS1 / hS0 (direction through the exp map of the old frame, position by
// translation) and, with cov_update, the scatter about the new mean is carried into the
// new frame by T = blkdiag(J, I3) and Sigma = (beta B + T C T^T / hW) / (beta a + bar0)
// replaces the covariance if it is SPD (else cholfail); the carried statistics become
// hS0 and T C T^T. The weight is left to the caller (it needs the cell's sum of bar0).
// When fac is given, the Cholesky factor of a replacing covariance (15 packed values) and
// the reciprocals of its diagonal (5) are written there too.
// With mir given, when the covariance is replaced the update also writes the EM part of the
// component's next E-step mirror there (floats 0-31, see mirror_core) from its own
// factorisation and frame, with the new weight pi_mir, returns its unshifted constant in
// c2_mir and sets mir_ok.
__device__ inline void component_map_update(double hS0, const double* hS1, const double* hS2, double hW,
                                            double beta, double bar0, const DevOpts& o, bool cov_update,
                                            const double mu_in[3], const double mux_in[3], double* mud,
                                            double* mux, double* cov, double* s0, double* s2, int& dead,
                                            int& cholfail, float* mir, double pi_mir, double& c2_mir, bool& mir_ok,
                                            double* fac = nullptr)
{
    mir_ok = false;
    if (!(bar0 > o.dead_threshold)) {
        dead = 1;
        *s0 = hS0;
        for (int q = 0; q < 15; ++q) s2[q] = hS2[q];
        return;
    }
    const double mu[3] = {mu_in[0], mu_in[1], mu_in[2]};
    double m[5];
    const double inv0 = 1.0 / hS0;
    for (int d = 0; d < 5; ++d) m[d] = hS1[d] * inv0;
    double Ro[9], Rn[9], mun[3];
    frame64(mu, Ro);
    const TangentRadius64 tr = tangent_radius64(m[0], m[1]);
    exp_map64(Ro, m[0], m[1], tr, mun);
    const double inn = 1.0 / sqrt(mun[0] * mun[0] + mun[1] * mun[1] + mun[2] * mun[2]);
    for (int i = 0; i < 3; ++i) mun[i] *= inn;
    double muxn[3];
    for (int i = 0; i < 3; ++i) {
        mud[i] = mun[i];
        muxn[i] = mux_in[i] + m[2 + i];
        mux[i] = muxn[i];
    }
    *s0 = hS0;
    if (!cov_update) return;
    frame64(mun, Rn);
    double J[4];
    transfer_jac64(Ro, Rn, m[0], m[1], tr, J);
    // scatter about the new mean in the old frame, then T C T^T with T = blkdiag(J, I3)
    double Cm[5][5];
    for (int d = 0; d < 5; ++d)
        for (int e = 0; e <= d; ++e) {
            const double v = hS2[tri(d, e)] - hS1[d] * hS1[e] * inv0;
            Cm[d][e] = v;
            Cm[e][d] = v;
        }
    double Tt[5][5];
    for (int b = 0; b < 5; ++b) {  // rows 0,1: J * C
        const double r0 = J[0] * Cm[0][b] + J[1] * Cm[1][b];
        const double r1 = J[2] * Cm[0][b] + J[3] * Cm[1][b];
        Tt[0][b] = r0;
        Tt[1][b] = r1;
        for (int a = 2; a < 5; ++a) Tt[a][b] = Cm[a][b];
    }
    for (int a = 0; a < 5; ++a) {  // columns 0,1: (J C) J^T
        const double c0 = Tt[a][0] * J[0] + Tt[a][1] * J[1];
        const double c1 = Tt[a][0] * J[2] + Tt[a][1] * J[3];
        Tt[a][0] = c0;
        Tt[a][1] = c1;
    }
    // the carried scatter first, so that it need not stay in registers through the
    // factorisation
    for (int d = 0; d < 5; ++d)
        for (int e = 0; e <= d; ++e) s2[tri(d, e)] = 0.5 * (Tt[d][e] + Tt[e][d]);
    double Sig[15], Lt[15];
    const double iden = 1.0 / (beta * o.prior_a + bar0), ihW = 1.0 / hW;
    for (int d = 0; d < 5; ++d)
        for (int e = 0; e <= d; ++e) {
            double v = 0.5 * (Tt[d][e] + Tt[e][d]) * ihW;
            if (d == e) v += beta * o.prior_b[d];
            Sig[tri(d, e)] = v * iden;
        }
    double Lti[5];
    if (chol64<5>(Sig, Lt, Lti)) {
        for (int q = 0; q < 15; ++q) cov[q] = Sig[q];
        if (fac) {
            for (int q = 0; q < 15; ++q) fac[q] = Lt[q];
            for (int d = 0; d < 5; ++d) fac[15 + d] = Lti[d];
        }
        if (mir) {
            double Li[15];
            mirror_core(pi_mir, Rn, muxn, Lt, Lti, mir, c2_mir, Li);
            mir[28] = mir[29] = mir[30] = mir[31] = 0.0f;
            mir_ok = true;
        }
    } else {
        cholfail = 1;
    }
}

// the same update without the mirror
__device__ __forceinline__ void component_map_update(double hS0, const double* hS1, const double* hS2, double hW,
                                                     double beta, double bar0, const DevOpts& o, bool cov_update,
                                                     const double mu_in[3], const double mux_in[3], double* mud,
                                                     double* mux, double* cov, double* s0, double* s2, int& dead,
                                                     int& cholfail, double* fac = nullptr)
{
    double c2;
    bool ok;
    component_map_update(hS0, hS1, hS2, hW, beta, bar0, o, cov_update, mu_in, mux_in, mud, mux, cov, s0, s2, dead,
                         cholfail, nullptr, 0.0, c2, ok, fac);
}

}  // namespace sdmm
