/*
 * sdmm_oracle.c -- plain, slow, FP64, single-threaded CPU reference ("the oracle")
 * for the spatio-directional mixture (SDMM) path of Dodik, Papas, Oztireli and
 * Mueller, "Path Guiding Using Spatio-Directional Mixture Models" (arXiv 2111.13094).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg load this library. The GPU library shares no code,
 * header, table or helper with it, and neither includes the other.
 *
 * What it computes, in the paper's order (section numbers are the paper's):
 *   - tangent-space log / exp maps of the sphere, with positions as translations
 *     (Sec. 3.1, log-map and exp-map equations, "Additional dimensions");
 *   - weighted sufficient statistics with responsibilities from tangent densities
 *     (Sec. 3.2, sufficient-statistics equation);
 *   - the M-step: weights, tangent-space mean update through the exp map, covariance
 *     computed in the old frame and carried to the new one by the first-order
 *     Jacobian (Sec. 3.2 mean update; Sec. 3.4 "Efficient tangent-space covariance
 *     update"; Appendix A); optionally the accurate covariance, from a second pass that
 *     takes the second moment in the new mean's tangent space (Sec. 3.2, "Sufficient
 *     statistics in tangent spaces");
 *   - Robbins-Monro averaging of the statistics and the normaliser across batches,
 *     and the MAP (Dirichlet / inverse-Wishart) updates (Sec. 4.3);
 *   - closed-form Gaussian conditioning on the position, the solid-angle pdf and
 *     sampling with the cut-locus discard (Sec. 3.1 density and sampling paragraphs,
 *     Sec. 3.2 first paragraph, Sec. 3.3);
 *   - the penalised log-likelihood that the MAP update maximises and its gradient;
 *   - product sampling of a conditioned radiance mixture with a conditioned BSDF mixture
 *     pruned to its two heaviest components (Sec. 3.4; Sec. 4.1 "Pruning before product
 *     sampling");
 *   - the spatial kD-tree: pre-subdivision, refinement of leaves with more than c
 *     samples at the mean of the axis of largest variance, copies of the mixture into
 *     new leaves, and initialisation of leaves that reached 16 samples (Sec. 4.2
 *     "Refinement of the spatial kD-tree", Sec. 4.3 "Initialization").
 *
 * Readings where the paper is silent or garbled (each one is listed with its reason
 * in the design notes): the frame R_mu is the branchless orthonormal basis of Duff et
 * al. 2017 with rows (t1, t2, mu); the solid-angle density divides the tangent density
 * by sinc|nu|; the corrected Jacobians of Appendix A; the Robbins-Monro weight eta_j
 * weights the new batch for every statistic; the prior strength is beta_j = eta_j / M_j
 * unless a fixed value is given; statistics are carried to the new frame after every
 * M-step with the first moment reset to zero; the prior is added after the transfer;
 * antipodal log-map input maps to (pi, 0); the accurate covariance pass takes its
 * responsibilities from the new weights and means with the previous covariances, its
 * covariance from that pass's S0 and S2, and is defined for batch steps (eta = 1) only;
 * a BSDF component is rotated to world with its tangent basis carried along, its
 * transfer Jacobian is taken at its conditioned offset, and the product pairs are
 * ordered 2k + j (radiance component k, j-th heaviest BSDF component).
 *
 * Layouts (shared as an interface with the GPU library, written independently):
 *   samples   float32 structure-of-arrays [7][N]: dir x,y,z, pos x,y,z, weight
 *   cov       5x5 symmetric packed lower triangle, row-major, index d(d+1)/2+e (d>=e),
 *             coordinate order (nu_u, nu_v, x, y, z)
 *   per cell  K components, component index fastest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define TRI(d, e) ((d) * ((d) + 1) / 2 + (e))
#define ORC_KMAX 64

/* per-cell status bits (the same values the GPU library reports) */
#define ORC_SKIPPED_FEW 1
#define ORC_SKIPPED_ZERO_W 2
#define ORC_BAD_INPUT 4
#define ORC_DEAD_COMPONENT 8
#define ORC_CHOL_FAIL_KEPT_PREV 16
#define ORC_BAD_PARAMS 32

typedef struct {
    int32_t K;
    int32_t iters;          /* E+M iterations on the given batch */
    int32_t eta_mode;       /* 0: eta_j = eta for j>0; 1: eta_j = (rm_beta*j+1)^-rm_alpha */
    int32_t prior_mode;     /* 0: beta_j = eta_j / M_j; 1: beta_j = prior_scale */
    int32_t estep_jacobian; /* 1: responsibilities from solid-angle densities */
    int32_t euclidean;      /* 1: the two directional coordinates are plain R^2 */
    int32_t min_samples;    /* cells with fewer positive-weight samples are skipped */
    int32_t accurate_sigma; /* 1: second moment re-taken in the new mean's tangent space */
    double eta, rm_alpha, rm_beta, prior_scale;
    double prior_q, prior_a, prior_b[5];
    double dead_threshold;
} orc_opts;

/* ------------------------------------------------------------------------- */
/* small dense helpers                                                        */
/* ------------------------------------------------------------------------- */

/* Cholesky factor of an n x n SPD matrix in packed lower storage. -1 if not SPD. */
static int chol_packed(int n, const double *A, double *L)
{
    for (int d = 0; d < n; ++d) {
        for (int e = 0; e <= d; ++e) {
            double s = A[TRI(d, e)];
            for (int f = 0; f < e; ++f) s -= L[TRI(d, f)] * L[TRI(e, f)];
            if (d == e) {
                if (!(s > 0.0) || !isfinite(s)) return -1;
                L[TRI(d, d)] = sqrt(s);
            } else {
                L[TRI(d, e)] = s / L[TRI(e, e)];
            }
        }
    }
    return 0;
}

/* solve L z = y for lower-triangular packed L */
static void forward_solve(int n, const double *L, const double *y, double *z)
{
    for (int d = 0; d < n; ++d) {
        double s = y[d];
        for (int e = 0; e < d; ++e) s -= L[TRI(d, e)] * z[e];
        z[d] = s / L[TRI(d, d)];
    }
}

/* full inverse of an SPD matrix from its Cholesky factor, dense n x n row-major */
static void spd_inverse(int n, const double *L, double *Ainv)
{
    double col[8], z[8], x[8];
    for (int j = 0; j < n; ++j) {
        for (int d = 0; d < n; ++d) col[d] = (d == j) ? 1.0 : 0.0;
        forward_solve(n, L, col, z);
        /* back substitution L^T x = z */
        for (int d = n - 1; d >= 0; --d) {
            double s = z[d];
            for (int e = d + 1; e < n; ++e) s -= L[TRI(e, d)] * x[e];
            x[d] = s / L[TRI(d, d)];
        }
        for (int d = 0; d < n; ++d) Ainv[d * n + j] = x[d];
    }
}

static double log_det_from_chol(int n, const double *L)
{
    double s = 0.0;
    for (int d = 0; d < n; ++d) s += log(L[TRI(d, d)]);
    return 2.0 * s;
}

/* ------------------------------------------------------------------------- */
/* tangent-space maps (Sec. 3.1)                                              */
/* ------------------------------------------------------------------------- */

/* Frame R_mu: rows (t1, t2, mu), so R_mu mu = (0,0,1). The paper only asks for "the
 * rotation that takes mu to +z"; this is the branchless basis of Duff et al. 2017. */
void orc_frame(const double mu[3], double R[9])
{
    double sgn = copysign(1.0, mu[2]);
    double a = -1.0 / (sgn + mu[2]);
    double b = mu[0] * mu[1] * a;
    R[0] = 1.0 + sgn * mu[0] * mu[0] * a;
    R[1] = sgn * b;
    R[2] = -sgn * mu[0];
    R[3] = b;
    R[4] = sgn + mu[1] * mu[1] * a;
    R[5] = -mu[1];
    R[6] = mu[0];
    R[7] = mu[1];
    R[8] = mu[2];
}

/* log map, Sec. 3.1: nu = (w'_x, w'_y) / sinc(acos w'_z) with w' = R w, written with
 * theta = atan2(|w'_xy|, w'_z) so that theta / sin(theta) = theta / |w'_xy|. */
void orc_log_map(const double R[9], const double w[3], double nu[2])
{
    double x = R[0] * w[0] + R[1] * w[1] + R[2] * w[2];
    double y = R[3] * w[0] + R[4] * w[1] + R[5] * w[2];
    double z = R[6] * w[0] + R[7] * w[1] + R[8] * w[2];
    double s = hypot(x, y);
    if (s > 0.0) {
        double th = atan2(s, z);
        nu[0] = th / s * x;
        nu[1] = th / s * y;
    } else if (z >= 0.0) {
        nu[0] = 0.0; /* w = mu */
        nu[1] = 0.0;
    } else {
        nu[0] = ORC_PI; /* antipode: the cut locus; reading (pi, 0) */
        nu[1] = 0.0;
    }
}

/* exp map, Sec. 3.1: w = R^-1 (nu sinc|nu|, cos|nu|) */
void orc_exp_map(const double R[9], const double nu[2], double w[3])
{
    double r = hypot(nu[0], nu[1]);
    double sc = (r > 0.0) ? sin(r) / r : 1.0;
    double v[3] = {nu[0] * sc, nu[1] * sc, cos(r)};
    for (int j = 0; j < 3; ++j) w[j] = R[j] * v[0] + R[3 + j] * v[1] + R[6 + j] * v[2];
}

/* (cos r - sinc r) / r^2, the scalar of the exp-map Jacobian (Appendix A) */
static double exp_jac_scalar(double r)
{
    if (r < 1e-2) {
        double r2 = r * r;
        return -1.0 / 3.0 + r2 / 30.0 - r2 * r2 / 840.0;
    }
    return (cos(r) - sin(r) / r) / (r * r);
}

/* d(nu sinc|nu|, cos|nu|)/d nu, a 3x2 matrix (Appendix A, with its two printed typos
 * corrected: off-diagonals are nu_x nu_y c and entry (2,2) is sinc + nu_y^2 c). */
static void exp_jac_local(const double nu[2], double M[6])
{
    double r = hypot(nu[0], nu[1]);
    double s = (r > 0.0) ? sin(r) / r : 1.0;
    double c = exp_jac_scalar(r);
    M[0] = s + nu[0] * nu[0] * c;
    M[1] = nu[0] * nu[1] * c;
    M[2] = nu[0] * nu[1] * c;
    M[3] = s + nu[1] * nu[1] * c;
    M[4] = -nu[0] * s;
    M[5] = -nu[1] * s;
}

/* First-order transfer between tangent spaces (Sec. 3.4): the Jacobian of
 * log_{mu_new} o exp_{mu} at nu = m, where mu_new = exp_mu(m). At that point
 * d log_{mu_new}/d w = rows (t1, t2) of R_{mu_new}, and d exp_mu/d nu = R_mu^T M(m). */
void orc_transfer_jacobian(const double mu[3], const double m[2], double J[4])
{
    double R[9], Rn[9], mun[3], M[6];
    orc_frame(mu, R);
    orc_exp_map(R, m, mun);
    double nn = sqrt(mun[0] * mun[0] + mun[1] * mun[1] + mun[2] * mun[2]);
    for (int i = 0; i < 3; ++i) mun[i] /= nn;
    orc_frame(mun, Rn);
    exp_jac_local(m, M);
    double RtM[6]; /* 3x2: R^T M */
    for (int j = 0; j < 3; ++j)
        for (int b = 0; b < 2; ++b) {
            double s = 0.0;
            for (int i = 0; i < 3; ++i) s += R[3 * i + j] * M[2 * i + b];
            RtM[2 * j + b] = s;
        }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double s = 0.0;
            for (int j = 0; j < 3; ++j) s += Rn[3 * a + j] * RtM[2 * j + b];
            J[2 * a + b] = s;
        }
}

/* ------------------------------------------------------------------------- */
/* per-component model pieces                                                 */
/* ------------------------------------------------------------------------- */

typedef struct {
    double R[9];
    double L[15];
    double logc; /* log pi - 0.5 log det Sigma - (5/2) log 2 pi */
    int ok;
} comp_t;

/* A component is usable when its weight is finite and non-negative, its means are
 * finite and its covariance is symmetric positive definite. */
static int component_ok(const double *pi, const double *mud, const double *mux, const double *cov,
                        double *L)
{
    if (!isfinite(*pi) || *pi < 0.0) return 0;
    for (int d = 0; d < 3; ++d)
        if (!isfinite(mud[d]) || !isfinite(mux[d])) return 0;
    return chol_packed(5, cov, L) == 0;
}

static int setup_components(int K, const double *pi, const double *mud, const double *mux,
                            const double *cov, comp_t *c)
{
    int bad = 0;
    for (int k = 0; k < K; ++k) {
        orc_frame(mud + 3 * k, c[k].R);
        c[k].ok = component_ok(pi + k, mud + 3 * k, mux + 3 * k, cov + 15 * k, c[k].L);
        if (!c[k].ok) {
            bad = 1;
            continue;
        }
        c[k].logc = log(pi[k]) - 0.5 * log_det_from_chol(5, c[k].L) - 2.5 * log(2.0 * ORC_PI);
    }
    return bad;
}

/* y = (log_mu w, p - mu_x), Sec. 3.1 "Additional dimensions" */
static void tangent_coords(const orc_opts *o, const comp_t *c, const double *mud, const double *mux,
                           const double w[3], const double p[3], double y[5])
{
    if (o->euclidean) {
        y[0] = w[0] - mud[0];
        y[1] = w[1] - mud[1];
    } else {
        orc_log_map(c->R, w, y);
    }
    for (int d = 0; d < 3; ++d) y[2 + d] = p[d] - mux[d];
}

/* log of the component density used in the E-step: the tangent density of Sec. 3.1,
 * or, with estep_jacobian, the solid-angle density (tangent density / sinc|nu|). */
static double comp_log_density(const orc_opts *o, const comp_t *c, const double y[5])
{
    double z[5];
    forward_solve(5, c->L, y, z);
    double q = 0.0;
    for (int d = 0; d < 5; ++d) q += z[d] * z[d];
    double l = c->logc - 0.5 * q;
    if (o->estep_jacobian && !o->euclidean) {
        double r = hypot(y[0], y[1]);
        if (r > 0.0) l -= log(sin(r) / r);
    }
    return l;
}

static int sample_is_bad(const float *smp, int64_t N, int64_t i)
{
    for (int a = 0; a < 7; ++a)
        if (!isfinite((double)smp[a * N + i])) return 1;
    return smp[6 * N + i] < 0.0f;
}

static void load_sample(const float *smp, int64_t N, int64_t i, double w[3], double p[3], double *wt)
{
    for (int d = 0; d < 3; ++d) {
        w[d] = (double)smp[d * N + i];
        p[d] = (double)smp[(3 + d) * N + i];
    }
    *wt = (double)smp[6 * N + i];
}

/* ------------------------------------------------------------------------- */
/* E-step statistics (Sec. 3.2)                                               */
/* ------------------------------------------------------------------------- */

/* Unnormalised statistics of samples [i0, i1) about the current parameters:
 * S0_k = sum w r, S1_k = sum w r y, S2_k = sum w r y y^T (packed), W = sum w,
 * M = #{w > 0}, LL = sum w log p(y). Returns status bits for bad input / params. */
int orc_cell_stats(const orc_opts *o, int32_t K, const float *smp, int64_t N, int64_t i0,
                   int64_t i1, const double *pi, const double *mud, const double *mux,
                   const double *cov, double *S0, double *S1, double *S2, double *W,
                   int64_t *M, double *LL)
{
    comp_t c[ORC_KMAX];
    double l[ORC_KMAX], y[ORC_KMAX][5];
    memset(S0, 0, sizeof(double) * K);
    memset(S1, 0, sizeof(double) * K * 5);
    memset(S2, 0, sizeof(double) * K * 15);
    *W = 0.0;
    *M = 0;
    *LL = 0.0;
    for (int64_t i = i0; i < i1; ++i)
        if (sample_is_bad(smp, N, i)) return ORC_BAD_INPUT;
    if (setup_components(K, pi, mud, mux, cov, c)) return ORC_BAD_PARAMS;
    for (int64_t i = i0; i < i1; ++i) {
        double w[3], p[3], wt;
        load_sample(smp, N, i, w, p, &wt);
        *W += wt;
        if (wt > 0.0) *M += 1;
        double lmax = -INFINITY;
        for (int k = 0; k < K; ++k) {
            tangent_coords(o, &c[k], mud + 3 * k, mux + 3 * k, w, p, y[k]);
            l[k] = comp_log_density(o, &c[k], y[k]);
            if (l[k] > lmax) lmax = l[k];
        }
        double den = 0.0;
        for (int k = 0; k < K; ++k) den += exp(l[k] - lmax);
        *LL += wt * (lmax + log(den));
        for (int k = 0; k < K; ++k) {
            double r = exp(l[k] - lmax) / den; /* responsibility */
            double wr = wt * r;
            S0[k] += wr;
            for (int d = 0; d < 5; ++d) {
                S1[5 * k + d] += wr * y[k][d];
                for (int e = 0; e <= d; ++e) S2[15 * k + TRI(d, e)] += wr * y[k][d] * y[k][e];
            }
        }
    }
    return 0;
}

/* responsibilities of one sample (for the "sum to one" pin) */
int orc_responsibilities(const orc_opts *o, int32_t K, const double w[3], const double p[3],
                         const double *pi, const double *mud, const double *mux,
                         const double *cov, double *r)
{
    comp_t c[ORC_KMAX];
    double l[ORC_KMAX], y[5];
    if (setup_components(K, pi, mud, mux, cov, c)) return ORC_BAD_PARAMS;
    double lmax = -INFINITY;
    for (int k = 0; k < K; ++k) {
        tangent_coords(o, &c[k], mud + 3 * k, mux + 3 * k, w, p, y);
        l[k] = comp_log_density(o, &c[k], y);
        if (l[k] > lmax) lmax = l[k];
    }
    double den = 0.0;
    for (int k = 0; k < K; ++k) den += exp(l[k] - lmax);
    for (int k = 0; k < K; ++k) r[k] = exp(l[k] - lmax) / den;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Robbins-Monro blend and MAP M-step (Sec. 3.2, 3.4, 4.3)                    */
/* ------------------------------------------------------------------------- */

double orc_eta(const orc_opts *o, int32_t j)
{
    if (j == 0) return 1.0;
    if (o->eta_mode == 0) return o->eta;
    return pow(o->rm_beta * (double)j + 1.0, -o->rm_alpha);
}

static int cell_mstep(const orc_opts *o, int K, int64_t M, double W, const double *S0,
                      const double *S1, const double *S2, double *pi, double *mud, double *mux,
                      double *cov, double *s0, double *s2, double *sw, int32_t *step)
{
    int status = 0;
    const int j = *step;
    const double eta = orc_eta(o, j);
    const double beta = (o->prior_mode == 0) ? eta / (double)M : o->prior_scale;

    /* Robbins-Monro averaging of S0, S1, S2 and the normaliser (Sec. 4.3). The carried
     * first moment is zero: it was taken about the mean it produced. */
    double hW = (j == 0) ? W : (1.0 - eta) * (*sw) + eta * W;
    double hS0[ORC_KMAX], hS1[ORC_KMAX][5], hS2[ORC_KMAX][15];
    for (int k = 0; k < K; ++k) {
        hS0[k] = (j == 0) ? S0[k] : (1.0 - eta) * s0[k] + eta * S0[k];
        for (int d = 0; d < 5; ++d) hS1[k][d] = (j == 0) ? S1[5 * k + d] : eta * S1[5 * k + d];
        for (int t = 0; t < 15; ++t)
            hS2[k][t] = (j == 0) ? S2[15 * k + t] : (1.0 - eta) * s2[15 * k + t] + eta * S2[15 * k + t];
    }

    double sum_bar0 = 0.0;
    for (int k = 0; k < K; ++k) sum_bar0 += hS0[k] / hW;

    for (int k = 0; k < K; ++k) {
        double bar0 = hS0[k] / hW;
        if (!(bar0 > o->dead_threshold)) {
            /* dead component: mean and covariance kept; its statistics are kept as blended */
            status |= ORC_DEAD_COMPONENT;
            s0[k] = hS0[k];
            for (int t = 0; t < 15; ++t) s2[15 * k + t] = hS2[k][t];
            continue;
        }
        double m[5];
        for (int d = 0; d < 5; ++d) m[d] = hS1[k][d] / hS0[k];

        /* mean update: directional part through the exp map of the old frame (Sec. 3.2),
         * positional part as a translation */
        double mu_old[3] = {mud[3 * k], mud[3 * k + 1], mud[3 * k + 2]};
        double mu_new[3];
        double J[4];
        if (o->euclidean) {
            mu_new[0] = mu_old[0] + m[0];
            mu_new[1] = mu_old[1] + m[1];
            mu_new[2] = mu_old[2];
            J[0] = 1.0; J[1] = 0.0; J[2] = 0.0; J[3] = 1.0;
        } else {
            double R[9];
            orc_frame(mu_old, R);
            orc_exp_map(R, m, mu_new);
            double nn = sqrt(mu_new[0] * mu_new[0] + mu_new[1] * mu_new[1] + mu_new[2] * mu_new[2]);
            for (int i = 0; i < 3; ++i) mu_new[i] /= nn;
            orc_transfer_jacobian(mu_old, m, J);
        }

        /* scatter about the new mean, still in the old frame (Sec. 3.2, params-from-stats) */
        double C[5][5];
        for (int d = 0; d < 5; ++d)
            for (int e = 0; e <= d; ++e) {
                double v = hS2[k][TRI(d, e)] - hS1[k][d] * hS1[k][e] / hS0[k];
                C[d][e] = v;
                C[e][d] = v;
            }
        /* first-order transfer to the new frame, T = blkdiag(J, I3) (Sec. 3.4) */
        double T[5][5] = {{0}};
        T[0][0] = J[0]; T[0][1] = J[1]; T[1][0] = J[2]; T[1][1] = J[3];
        T[2][2] = 1.0; T[3][3] = 1.0; T[4][4] = 1.0;
        double TC[5][5], Cn[5][5];
        for (int a = 0; a < 5; ++a)
            for (int b = 0; b < 5; ++b) {
                double s = 0.0;
                for (int q = 0; q < 5; ++q) s += T[a][q] * C[q][b];
                TC[a][b] = s;
            }
        for (int a = 0; a < 5; ++a)
            for (int b = 0; b < 5; ++b) {
                double s = 0.0;
                for (int q = 0; q < 5; ++q) s += TC[a][q] * T[b][q];
                Cn[a][b] = s;
            }

        /* MAP covariance (Sec. 4.3): (beta B + S2/W) / (beta a + S0/W), B diagonal */
        double Sig[15], Lt[15];
        double den = beta * o->prior_a + bar0;
        for (int d = 0; d < 5; ++d)
            for (int e = 0; e <= d; ++e) {
                double v = 0.5 * (Cn[d][e] + Cn[e][d]) / hW;
                if (d == e) v += beta * o->prior_b[d];
                Sig[TRI(d, e)] = v / den;
            }

        for (int i = 0; i < 3; ++i) {
            mud[3 * k + i] = mu_new[i];
            mux[3 * k + i] += m[2 + i];
        }
        if (chol_packed(5, Sig, Lt) == 0) {
            memcpy(cov + 15 * k, Sig, sizeof(Sig));
        } else {
            status |= ORC_CHOL_FAIL_KEPT_PREV;
        }
        /* carried statistics, now about the new mean in the new frame */
        s0[k] = hS0[k];
        for (int d = 0; d < 5; ++d)
            for (int e = 0; e <= d; ++e) s2[15 * k + TRI(d, e)] = 0.5 * (Cn[d][e] + Cn[e][d]);
    }

    /* MAP weights (Sec. 4.3) */
    double wden = (double)K * beta * o->prior_q + sum_bar0;
    for (int k = 0; k < K; ++k) pi[k] = (beta * o->prior_q + hS0[k] / hW) / wden;

    *sw = hW;
    *step = j + 1;
    return status;
}

/* Gate, Sec. 4.2: a cell is updated only with at least min_samples vertices. */
static int gate(const orc_opts *o, int K, const float *smp, int64_t N, int64_t i0, int64_t i1,
                const double *pi, const double *mud, const double *mux, const double *cov,
                int64_t *M, double *W)
{
    for (int64_t i = i0; i < i1; ++i)
        if (sample_is_bad(smp, N, i)) return ORC_BAD_INPUT;
    for (int k = 0; k < K; ++k) {
        double L[15];
        if (!component_ok(pi + k, mud + 3 * k, mux + 3 * k, cov + 15 * k, L)) return ORC_BAD_PARAMS;
    }
    *M = 0;
    *W = 0.0;
    for (int64_t i = i0; i < i1; ++i) {
        double wt = (double)smp[6 * N + i];
        *W += wt;
        if (wt > 0.0) *M += 1;
    }
    if (*M < o->min_samples) return ORC_SKIPPED_FEW;
    if (!(*W > 0.0)) return ORC_SKIPPED_ZERO_W;
    return 0;
}

/* Accurate covariance update (Sec. 3.2, "Sufficient statistics in tangent spaces"). The
 * second moment that sets the new covariance is taken in the tangent space of the new
 * mean, with responsibilities from the component densities in that tangent space. Once
 * the M-step has produced the new weights and means, a second E-step runs under
 * (pi^, mu^, Sigma), Sigma being the covariance before the step (the only one known),
 * giving S0'_k = sum w r', S2'_k = sum w r' y^ y^^T with y^ = (log_{mu^} w, p - mu^_x),
 * and Sigma^_k = (beta B + S2'_k / W) / (beta a + S0'_k / W): the covariance about the new
 * mean, without a mean subtracted. Defined for batch steps (eta = 1), where no carried
 * statistic needs moving. Components dead in the M-step keep what it left; a component
 * whose S0'/W is at or below the dead threshold keeps its covariance and flags the cell
 * as dead; a covariance that is not SPD keeps the previous one and flags the cell. For
 * every component not dead in the M-step the carried S0 and S2 become S0' and S2'. */
static int accurate_sigma_pass(const orc_opts *o, int K, const float *smp, int64_t N, int64_t i0,
                               int64_t i1, const double *S0, double W, int64_t M, const double *pi,
                               const double *mud, const double *mux, const double *cov0, double *cov,
                               double *s0, double *s2)
{
    double T0[ORC_KMAX], T1[ORC_KMAX * 5], T2[ORC_KMAX * 15], W2, LL;
    int64_t M2;
    int status = 0;
    /* the E-step under the new weights and means and the previous covariances */
    memcpy(cov, cov0, sizeof(double) * 15 * K);
    if (orc_cell_stats(o, K, smp, N, i0, i1, pi, mud, mux, cov, T0, T1, T2, &W2, &M2, &LL)) return ORC_BAD_PARAMS;
    const double beta = (o->prior_mode == 0) ? 1.0 / (double)M : o->prior_scale;
    for (int k = 0; k < K; ++k) {
        if (!(S0[k] / W > o->dead_threshold)) continue; /* dead in the M-step */
        s0[k] = T0[k];
        memcpy(s2 + 15 * k, T2 + 15 * k, sizeof(double) * 15);
        const double bar0 = T0[k] / W2;
        if (!(bar0 > o->dead_threshold)) {
            status |= ORC_DEAD_COMPONENT;
            continue;
        }
        double Sig[15], Lt[15];
        const double den = beta * o->prior_a + bar0;
        for (int d = 0; d < 5; ++d)
            for (int e = 0; e <= d; ++e) {
                double v = T2[15 * k + TRI(d, e)] / W2;
                if (d == e) v += beta * o->prior_b[d];
                Sig[TRI(d, e)] = v / den;
            }
        if (chol_packed(5, Sig, Lt) == 0)
            memcpy(cov + 15 * k, Sig, sizeof(Sig));
        else
            status |= ORC_CHOL_FAIL_KEPT_PREV;
    }
    return status;
}

/* One E+M step of one cell on its samples [i0, i1): gate, statistics, M-step (and the
 * accurate covariance pass when asked for). Returns the status bits; stops the cell
 * (*stop = 1) when it is gated or its statistics are not finite. */
static int cell_batch_step(const orc_opts *o, int K, const float *smp, int64_t N, int64_t i0, int64_t i1,
                           double *pi, double *mud, double *mux, double *cov, double *s0, double *s2, double *sw,
                           int32_t *step, int *stop)
{
    double S0[ORC_KMAX], S1[ORC_KMAX * 5], S2[ORC_KMAX * 15];
    double cov0[ORC_KMAX * 15];
    int64_t M;
    double W, LL;
    *stop = 0;
    int g = gate(o, K, smp, N, i0, i1, pi, mud, mux, cov, &M, &W);
    if (g) {
        *stop = 1;
        return g;
    }
    orc_cell_stats(o, K, smp, N, i0, i1, pi, mud, mux, cov, S0, S1, S2, &W, &M, &LL);
    /* statistics that are not finite (e.g. every component has zero weight) leave the cell
     * untouched and are reported like bad input */
    int finite = isfinite(W);
    for (int t = 0; t < K && finite; ++t) {
        finite = isfinite(S0[t]);
        for (int d = 0; d < 5; ++d) finite = finite && isfinite(S1[5 * t + d]);
        for (int d = 0; d < 15; ++d) finite = finite && isfinite(S2[15 * t + d]);
    }
    if (!finite) {
        *stop = 1;
        return ORC_BAD_INPUT;
    }
    if (o->accurate_sigma) memcpy(cov0, cov, sizeof(double) * 15 * K);
    int ms = cell_mstep(o, K, M, W, S0, S1, S2, pi, mud, mux, cov, s0, s2, sw, step);
    if (o->accurate_sigma) {
        /* the first-order covariance of the M-step is replaced by the second pass, and so
         * is its SPD verdict */
        ms &= ~ORC_CHOL_FAIL_KEPT_PREV;
        ms |= accurate_sigma_pass(o, K, smp, N, i0, i1, S0, W, M, pi, mud, mux, cov0, cov, s0, s2);
    }
    return ms;
}

/* the offsets must partition a prefix of the sample array: non-decreasing, from >= 0 to
 * <= N. An array that is not is rejected as a whole: every cell reports bad input and
 * nothing changes (a decreasing entry says the batch itself is malformed). */
static int offsets_valid(int32_t n_cells, const int64_t *offsets, int64_t N, int32_t *status)
{
    int ok = n_cells == 0 || (offsets[0] >= 0 && offsets[n_cells] <= N);
    for (int32_t c = 0; c < n_cells && ok; ++c) ok = offsets[c + 1] >= offsets[c];
    if (!ok)
        for (int32_t c = 0; c < n_cells; ++c) status[c] = ORC_BAD_INPUT;
    return ok;
}

/* Fit: o->iters E+M iterations of every cell on the given batch. Parameters and the
 * averaged statistics are updated in place; status[c] receives the OR of the cell's
 * status bits over the iterations. */
int orc_fit(const orc_opts *o, int32_t n_cells, const int64_t *offsets, const float *smp, int64_t N,
            double *pi, double *mud, double *mux, double *cov, double *s0, double *s2, double *sw,
            int32_t *step, int32_t *status)
{
    const int K = o->K;
    if (K < 1 || K > ORC_KMAX) return -1;
    /* the accurate covariance update is defined for batch steps */
    if (o->accurate_sigma && !(o->eta_mode == 0 && o->eta == 1.0)) return -2;
    if (!offsets_valid(n_cells, offsets, N, status)) return 0;
    /* cells are independent (Sec. 4.2); a build with OpenMP (the all-cores CPU baseline)
     * spreads them over threads, each cell's arithmetic unchanged */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int32_t c = 0; c < n_cells; ++c) {
        const int64_t ck = (int64_t)c * K;
        status[c] = 0;
        for (int it = 0; it < o->iters; ++it) {
            int stop;
            status[c] |= cell_batch_step(o, K, smp, N, offsets[c], offsets[c + 1], pi + ck, mud + 3 * ck,
                                         mux + 3 * ck, cov + 15 * ck, s0 + ck, s2 + 15 * ck, sw + c, step + c,
                                         &stop);
            if (stop) break;
        }
    }
    return 0;
}

/* Stepwise EM, the per-sample alternative of Sec. 6 ("Mini-batch EM versus stepwise EM";
 * Cappe and Moulines 2009, weighted as in Vorba et al. 2014): each sample with positive
 * weight, in index order, is a mini-batch of one. Its statistics are taken under the
 * current parameters, blended with eta_j for the cell's sample counter j, and the MAP
 * M-step follows with M = 1 (so beta_j = eta_j unless fixed), including the first-order
 * transport of the carried second moment into the new frame. A cell whose state is fresh
 * (step 0) first takes one mini-batch step over its samples: the blend needs statistics
 * to start from. The cell gate applies to the whole batch before each pass; o->iters
 * passes over the samples. The accurate covariance update is not defined here (-2). */
int orc_fit_stepwise(const orc_opts *o, int32_t n_cells, const int64_t *offsets, const float *smp, int64_t N,
                     double *pi, double *mud, double *mux, double *cov, double *s0, double *s2, double *sw,
                     int32_t *step, int32_t *status)
{
    const int K = o->K;
    if (K < 1 || K > ORC_KMAX) return -1;
    if (o->accurate_sigma) return -2;
    if (!offsets_valid(n_cells, offsets, N, status)) return 0;
    double S0[ORC_KMAX], S1[ORC_KMAX * 5], S2[ORC_KMAX * 15];
    for (int32_t c = 0; c < n_cells; ++c) {
        const int64_t i0 = offsets[c], i1 = offsets[c + 1];
        const int64_t ck = (int64_t)c * K;
        double *P = pi + ck, *D = mud + 3 * ck, *X = mux + 3 * ck, *V = cov + 15 * ck;
        status[c] = 0;
        for (int it = 0; it < o->iters; ++it) {
            int stop = 0;
            if (step[c] == 0) {
                status[c] |= cell_batch_step(o, K, smp, N, i0, i1, P, D, X, V, s0 + ck, s2 + 15 * ck, sw + c,
                                             step + c, &stop);
                if (stop) break;
                continue;
            }
            int64_t M;
            double W, LL;
            int g = gate(o, K, smp, N, i0, i1, P, D, X, V, &M, &W);
            if (g) {
                status[c] |= g;
                break;
            }
            for (int64_t i = i0; i < i1 && !stop; ++i) {
                if (!(smp[6 * N + i] > 0.0f)) continue;
                orc_cell_stats(o, K, smp, N, i, i + 1, P, D, X, V, S0, S1, S2, &W, &M, &LL);
                int finite = isfinite(W);
                for (int t = 0; t < K && finite; ++t) {
                    finite = isfinite(S0[t]);
                    for (int d = 0; d < 5; ++d) finite = finite && isfinite(S1[5 * t + d]);
                    for (int d = 0; d < 15; ++d) finite = finite && isfinite(S2[15 * t + d]);
                }
                if (!finite) {
                    status[c] |= ORC_BAD_INPUT;
                    stop = 1;
                    break;
                }
                status[c] |= cell_mstep(o, K, 1, W, S0, S1, S2, P, D, X, V, s0 + ck, s2 + 15 * ck, sw + c,
                                        step + c);
            }
            if (stop) break;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* penalised log-likelihood and its gradient                                  */
/* ------------------------------------------------------------------------- */

/* F = sum_i (w_i/W) log sum_k pi_k N5(y_ik; 0, Sigma_k)
 *     + sum_k [ beta q log pi_k - (beta a / 2) log det Sigma_k - (beta / 2) tr(B Sigma_k^-1) ],
 * the function whose maximiser is the MAP update of Sec. 4.3 (Dirichlet prior on the
 * weights, inverse-Wishart prior on the covariances, no prior on the means). */
double orc_objective(const orc_opts *o, int32_t K, const float *smp, int64_t N, int64_t i0,
                     int64_t i1, const double *pi, const double *mud, const double *mux,
                     const double *cov, double beta)
{
    double S0[ORC_KMAX], S1[ORC_KMAX * 5], S2[ORC_KMAX * 15], W, LL;
    int64_t M;
    if (orc_cell_stats(o, K, smp, N, i0, i1, pi, mud, mux, cov, S0, S1, S2, &W, &M, &LL)) return NAN;
    double F = LL / W;
    for (int k = 0; k < K; ++k) {
        double L[15], Si[25];
        chol_packed(5, cov + 15 * k, L);
        spd_inverse(5, L, Si);
        double tr = 0.0;
        for (int d = 0; d < 5; ++d) tr += o->prior_b[d] * Si[d * 5 + d];
        F += beta * o->prior_q * log(pi[k]) - 0.5 * beta * o->prior_a * log_det_from_chol(5, L) -
             0.5 * beta * tr;
    }
    return F;
}

/* d nu / d delta for nu = log_{mu(delta)}(w), mu(delta) = exp_mu(delta), frame rebuilt by
 * orc_frame at mu(delta); evaluated at delta = 0 by the chain rule through the frame. */
static void dlog_ddelta(const double mu[3], const double R[9], const double w[3], double D[4])
{
    const double sgn = copysign(1.0, mu[2]);
    const double a = -1.0 / (sgn + mu[2]);
    const double a2 = a * a;
    const double nx = mu[0], ny = mu[1];
    /* partial derivatives of the frame rows with respect to mu (3x3 each, row-major) */
    const double db[3] = {ny * a, nx * a, nx * ny * a2};
    const double dt1[9] = {2.0 * sgn * nx * a, 0.0, sgn * nx * nx * a2,
                           sgn * db[0], sgn * db[1], sgn * db[2],
                           -sgn, 0.0, 0.0};
    const double dt2[9] = {db[0], db[1], db[2],
                           0.0, 2.0 * ny * a, ny * ny * a2,
                           0.0, -1.0, 0.0};
    double x = R[0] * w[0] + R[1] * w[1] + R[2] * w[2];
    double y = R[3] * w[0] + R[4] * w[1] + R[5] * w[2];
    double z = R[6] * w[0] + R[7] * w[1] + R[8] * w[2];
    double s = hypot(x, y);
    double th = atan2(s, z);
    for (int jj = 0; jj < 2; ++jj) {
        const double *dmu = R + 3 * jj; /* d mu / d delta_j at 0 = t_j */
        double dx = 0.0, dy = 0.0, dz = 0.0;
        for (int i = 0; i < 3; ++i) {
            double g1 = 0.0, g2 = 0.0;
            for (int q = 0; q < 3; ++q) {
                g1 += dt1[3 * i + q] * dmu[q];
                g2 += dt2[3 * i + q] * dmu[q];
            }
            dx += g1 * w[i];
            dy += g2 * w[i];
            dz += dmu[i] * w[i];
        }
        double f, df;
        if (s > 1e-6) {
            double ds = (x * dx + y * dy) / s;
            double dth = (z * ds - s * dz) / (s * s + z * z);
            f = th / s;
            df = dth / s - th * ds / (s * s);
        } else {
            f = 1.0; /* theta/s -> 1; its first-order change is O(theta) -> dropped */
            df = 0.0;
        }
        D[0 * 2 + jj] = df * x + f * dx;
        D[1 * 2 + jj] = df * y + f * dy;
    }
}

/* Gradient of F at the current parameters with respect to the weight logits
 * (pi = softmax(alpha)), the positional means, a tangent perturbation delta of the
 * directional mean (mu(delta) = exp_mu(delta)), and the Cholesky factor L of Sigma
 * (packed lower). Outputs per component: g_alpha[K], g_mux[3K], g_delta[2K], g_L[15K]. */
int orc_grad(const orc_opts *o, int32_t K, const float *smp, int64_t N, int64_t i0, int64_t i1,
             const double *pi, const double *mud, const double *mux, const double *cov, double beta,
             double *g_alpha, double *g_mux, double *g_delta, double *g_L)
{
    double S0[ORC_KMAX], S1[ORC_KMAX * 5], S2[ORC_KMAX * 15], W, LL;
    int64_t M;
    int st = orc_cell_stats(o, K, smp, N, i0, i1, pi, mud, mux, cov, S0, S1, S2, &W, &M, &LL);
    if (st) return st;
    comp_t c[ORC_KMAX];
    setup_components(K, pi, mud, mux, cov, c);
    double Si[ORC_KMAX][25];
    double sum0 = 0.0;
    for (int k = 0; k < K; ++k) {
        spd_inverse(5, c[k].L, Si[k]);
        sum0 += S0[k] / W;
    }
    for (int k = 0; k < K; ++k) {
        double b0 = S0[k] / W;
        g_alpha[k] = b0 + beta * o->prior_q - pi[k] * (sum0 + K * beta * o->prior_q);
        /* d/d mu_x: [Sigma^-1 S1bar]_x */
        for (int d = 0; d < 3; ++d) {
            double s = 0.0;
            for (int e = 0; e < 5; ++e) s += Si[k][(2 + d) * 5 + e] * S1[5 * k + e] / W;
            g_mux[3 * k + d] = s;
        }
        /* G = 1/2 Sigma^-1 (S2bar + beta B) Sigma^-1 - 1/2 (S0bar + beta a) Sigma^-1 */
        double A[25], G[25];
        for (int d = 0; d < 5; ++d)
            for (int e = 0; e < 5; ++e) {
                int dd = d > e ? d : e, ee = d > e ? e : d;
                A[d * 5 + e] = S2[15 * k + TRI(dd, ee)] / W + ((d == e) ? beta * o->prior_b[d] : 0.0);
            }
        for (int d = 0; d < 5; ++d)
            for (int e = 0; e < 5; ++e) {
                double s = 0.0;
                for (int p = 0; p < 5; ++p)
                    for (int q = 0; q < 5; ++q) s += Si[k][d * 5 + p] * A[p * 5 + q] * Si[k][q * 5 + e];
                G[d * 5 + e] = 0.5 * s - 0.5 * (b0 + beta * o->prior_a) * Si[k][d * 5 + e];
            }
        /* dF/dL = tril(2 G L) */
        for (int d = 0; d < 5; ++d)
            for (int e = 0; e <= d; ++e) {
                double s = 0.0;
                for (int p = e; p < 5; ++p) s += G[d * 5 + p] * c[k].L[TRI(p, e)];
                g_L[15 * k + TRI(d, e)] = 2.0 * s;
            }
        g_delta[2 * k] = 0.0;
        g_delta[2 * k + 1] = 0.0;
    }
    /* d/d delta: -sum_i (w_i/W) r_ik (d nu_ik/d delta)^T [Sigma_k^-1 y_ik]_nu */
    double l[ORC_KMAX], y[ORC_KMAX][5];
    for (int64_t i = i0; i < i1; ++i) {
        double w[3], p[3], wt;
        load_sample(smp, N, i, w, p, &wt);
        if (wt == 0.0) continue;
        double lmax = -INFINITY;
        for (int k = 0; k < K; ++k) {
            tangent_coords(o, &c[k], mud + 3 * k, mux + 3 * k, w, p, y[k]);
            l[k] = comp_log_density(o, &c[k], y[k]);
            if (l[k] > lmax) lmax = l[k];
        }
        double den = 0.0;
        for (int k = 0; k < K; ++k) den += exp(l[k] - lmax);
        for (int k = 0; k < K; ++k) {
            double wr = wt / W * exp(l[k] - lmax) / den;
            double u0 = 0.0, u1 = 0.0;
            for (int e = 0; e < 5; ++e) {
                u0 += Si[k][0 * 5 + e] * y[k][e];
                u1 += Si[k][1 * 5 + e] * y[k][e];
            }
            double D[4];
            if (o->euclidean) {
                D[0] = -1.0; D[1] = 0.0; D[2] = 0.0; D[3] = -1.0;
            } else {
                dlog_ddelta(mud + 3 * k, c[k].R, w, D);
            }
            g_delta[2 * k] -= wr * (D[0] * u0 + D[2] * u1);
            g_delta[2 * k + 1] -= wr * (D[1] * u0 + D[3] * u1);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* conditioning, pdf and sampling (Sec. 3.1, 3.2, 3.3)                        */
/* ------------------------------------------------------------------------- */

/* Closed-form conditioning of one cell's joint mixture on the position x:
 * pi'_k ∝ pi_k N3(x - mu_x; 0, Sigma_xx), m_k = Sigma_nx Sigma_xx^-1 (x - mu_x),
 * Sigma'_k = Sigma_nn - Sigma_nx Sigma_xx^-1 Sigma_xn (packed 2x2). */
int orc_condition(int32_t K, const double *pi, const double *mux, const double *cov,
                  const double x[3], double *pic, double *m, double *Sc)
{
    double lw[ORC_KMAX], lmax = -INFINITY;
    for (int k = 0; k < K; ++k) {
        const double *S = cov + 15 * k;
        double Sxx[6], Lxx[6], Sxxi[9];
        for (int d = 0; d < 3; ++d)
            for (int e = 0; e <= d; ++e) Sxx[TRI(d, e)] = S[TRI(2 + d, 2 + e)];
        if (chol_packed(3, Sxx, Lxx) != 0) return -1;
        spd_inverse(3, Lxx, Sxxi);
        double dx[3], u[3];
        for (int d = 0; d < 3; ++d) dx[d] = x[d] - mux[3 * k + d];
        forward_solve(3, Lxx, dx, u);
        double q = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        lw[k] = log(pi[k]) - 0.5 * q - 0.5 * log_det_from_chol(3, Lxx) - 1.5 * log(2.0 * ORC_PI);
        if (lw[k] > lmax) lmax = lw[k];
        /* A = Sigma_nx Sigma_xx^-1 (2x3); Sigma_nx[a][d] = S[TRI(2+d, a)] */
        double A[6];
        for (int a = 0; a < 2; ++a)
            for (int d = 0; d < 3; ++d) {
                double s = 0.0;
                for (int e = 0; e < 3; ++e) s += S[TRI(2 + e, a)] * Sxxi[e * 3 + d];
                A[3 * a + d] = s;
            }
        for (int a = 0; a < 2; ++a) m[2 * k + a] = A[3 * a] * dx[0] + A[3 * a + 1] * dx[1] + A[3 * a + 2] * dx[2];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b <= a; ++b) {
                double s = S[TRI(a, b)];
                for (int d = 0; d < 3; ++d) s -= A[3 * a + d] * S[TRI(2 + d, b)];
                Sc[3 * k + TRI(a, b)] = s;
            }
    }
    double den = 0.0;
    for (int k = 0; k < K; ++k) den += exp(lw[k] - lmax);
    for (int k = 0; k < K; ++k) pic[k] = exp(lw[k] - lmax) / den;
    return 0;
}

/* Solid-angle pdf of the conditioned mixture (Sec. 3.1 mixture pdf), with the
 * change of variables dividing by sinc|nu| and a zero contribution at or beyond the
 * cut locus |nu| >= pi (1 - 1e-6). */
double orc_pdf_conditioned(int32_t K, const double *mud, const double *pic, const double *m,
                           const double *Sc, const double w[3])
{
    double p = 0.0;
    for (int k = 0; k < K; ++k) {
        if (pic[k] == 0.0) continue;
        double R[9], nu[2], L[3], d[2], z[2];
        orc_frame(mud + 3 * k, R);
        orc_log_map(R, w, nu);
        double r = hypot(nu[0], nu[1]);
        if (r >= ORC_PI * (1.0 - 1e-6)) continue;
        if (chol_packed(2, Sc + 3 * k, L) != 0) continue;
        d[0] = nu[0] - m[2 * k];
        d[1] = nu[1] - m[2 * k + 1];
        forward_solve(2, L, d, z);
        double q = z[0] * z[0] + z[1] * z[1];
        double pt = exp(-0.5 * q) / (2.0 * ORC_PI * L[0] * L[2]);
        double sinc = (r > 0.0) ? sin(r) / r : 1.0;
        p += pic[k] * pt / sinc;
    }
    return p;
}

/* Conditioned pdf for many (query, direction) pairs: query q lies in cell qcell[q];
 * directions dirs[(q*nd + t)*3 ...] (array of structures, 3 doubles). */
int orc_pdf(int32_t K, const double *pi, const double *mud, const double *mux, const double *cov,
            int64_t nq, const double *qpos, const int32_t *qcell, int32_t nd, const double *dirs,
            double *pdf_out)
{
    double pic[ORC_KMAX], m[2 * ORC_KMAX], Sc[3 * ORC_KMAX];
    for (int64_t q = 0; q < nq; ++q) {
        int64_t ck = (int64_t)qcell[q] * K;
        if (orc_condition(K, pi + ck, mux + 3 * ck, cov + 15 * ck, qpos + 3 * q, pic, m, Sc)) return -1;
        for (int t = 0; t < nd; ++t)
            pdf_out[q * nd + t] = orc_pdf_conditioned(K, mud + 3 * ck, pic, m, Sc, dirs + 3 * (q * nd + t));
    }
    return 0;
}

/* Sampling (Sec. 3.1): component by the CDF of pi' (lowest index on ties), nu from the
 * component's conditional Gaussian by Box-Muller with u1 mapped to (0,1], discard when
 * |nu| >= pi, w = exp_mu(nu), and the pdf of the whole conditioned mixture at w.
 * uniforms[(q*ns + t)*3 + {0,1,2}] in [0,1). Invalid draws give dir 0, pdf 0, valid 0. */
int orc_sample(int32_t K, const double *pi, const double *mud, const double *mux, const double *cov,
               int64_t nq, const double *qpos, const int32_t *qcell, int32_t ns,
               const double *uniforms, double *dirs_out, double *pdf_out, int32_t *comp_out,
               uint8_t *valid_out)
{
    double pic[ORC_KMAX], m[2 * ORC_KMAX], Sc[3 * ORC_KMAX];
    for (int64_t q = 0; q < nq; ++q) {
        int64_t ck = (int64_t)qcell[q] * K;
        if (orc_condition(K, pi + ck, mux + 3 * ck, cov + 15 * ck, qpos + 3 * q, pic, m, Sc)) return -1;
        for (int t = 0; t < ns; ++t) {
            const double *u = uniforms + 3 * (q * ns + t);
            int64_t o = q * ns + t;
            int sel = -1;
            double cdf = 0.0;
            for (int k = 0; k < K; ++k) {
                cdf += pic[k];
                if (u[0] < cdf) {
                    sel = k;
                    break;
                }
            }
            if (sel < 0)
                for (int k = K - 1; k >= 0; --k)
                    if (pic[k] > 0.0) {
                        sel = k;
                        break;
                    }
            comp_out[o] = sel;
            double L[3];
            chol_packed(2, Sc + 3 * sel, L);
            double rad = sqrt(-2.0 * log(1.0 - u[1]));
            double z0 = rad * cos(2.0 * ORC_PI * u[2]), z1 = rad * sin(2.0 * ORC_PI * u[2]);
            double nu[2] = {m[2 * sel] + L[0] * z0, m[2 * sel + 1] + L[1] * z0 + L[2] * z1};
            if (hypot(nu[0], nu[1]) >= ORC_PI) {
                valid_out[o] = 0;
                pdf_out[o] = 0.0;
                dirs_out[3 * o] = dirs_out[3 * o + 1] = dirs_out[3 * o + 2] = 0.0;
                continue;
            }
            double R[9], w[3];
            orc_frame(mud + 3 * (ck + sel), R);
            orc_exp_map(R, nu, w);
            valid_out[o] = 1;
            for (int d = 0; d < 3; ++d) dirs_out[3 * o + d] = w[d];
            pdf_out[o] = orc_pdf_conditioned(K, mud + 3 * ck, pic, m, Sc, w);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* product sampling with a conditioned BSDF mixture (Sec. 3.4; the pruning of   */
/* Sec. 4.1)                                                                  */
/* ------------------------------------------------------------------------- */

/* Derivative of the log map with respect to the frame coordinates p = R w of a unit
 * vector, a 2x3 matrix. With s = |(p_x, p_y)|, theta = atan2(s, p_z), f = theta / s and
 * nu = f (p_x, p_y): on the unit sphere d f/d p_x = p_x g, d f/d p_y = p_y g with
 * g = (p_z - f) / s^2, and d f/d p_z = -1. Near the mean g -> -2/3 - theta^2 / 5. */
static void log_jac_local(const double p[3], double Jl[6])
{
    double s = hypot(p[0], p[1]);
    double th = atan2(s, p[2]);
    double f = (s > 0.0) ? th / s : 1.0;
    double g = (s > 1e-3) ? (p[2] - f) / (s * s) : -2.0 / 3.0 - th * th / 5.0;
    Jl[0] = f + p[0] * p[0] * g;
    Jl[1] = p[0] * p[1] * g;
    Jl[2] = -p[0];
    Jl[3] = p[0] * p[1] * g;
    Jl[4] = f + p[1] * p[1] * g;
    Jl[5] = -p[1];
}

/* A component centred at offset m2 in the tangent space of mu2, seen from the tangent
 * space of mu1 (Sec. 3.4): its centre a = log_{mu1}(exp_{mu2}(m2)) and the Jacobian J of
 * log_{mu1} o exp_{mu2} at m2, the first-order map of its covariance (J Sigma J^T).
 * The Jacobian is d log / d w at the centre times d exp / d nu at m2 (Appendix A). */
void orc_pair_transfer(const double mu1[3], const double mu2[3], const double m2[2], double a[2], double J[4])
{
    double R1[9], R2[9], w[3], p[3], M[6], Jl[6];
    orc_frame(mu1, R1);
    orc_frame(mu2, R2);
    orc_exp_map(R2, m2, w);
    orc_log_map(R1, w, a);
    for (int i = 0; i < 3; ++i) p[i] = R1[3 * i] * w[0] + R1[3 * i + 1] * w[1] + R1[3 * i + 2] * w[2];
    log_jac_local(p, Jl);
    exp_jac_local(m2, M);
    /* d w / d nu = R2^T M (3x2); d p / d nu = R1 R2^T M */
    double D[6];
    for (int j = 0; j < 3; ++j)
        for (int b = 0; b < 2; ++b) {
            double s = 0.0;
            for (int i = 0; i < 3; ++i) s += R2[3 * i + j] * M[2 * i + b];
            D[2 * j + b] = s;
        }
    double P[6];
    for (int i = 0; i < 3; ++i)
        for (int b = 0; b < 2; ++b) P[2 * i + b] = R1[3 * i] * D[b] + R1[3 * i + 1] * D[2 + b] + R1[3 * i + 2] * D[4 + b];
    for (int r = 0; r < 2; ++r)
        for (int b = 0; b < 2; ++b) J[2 * r + b] = Jl[3 * r] * P[b] + Jl[3 * r + 1] * P[2 + b] + Jl[3 * r + 2] * P[4 + b];
}

/* A tangent-space component rotated by the local-to-world rotation F (world = F local):
 * the mean becomes F mu; the frame of F mu differs from F applied to the frame of mu by
 * a rotation Q inside the tangent plane, Q_ij = t_i(F mu) . F t_j(mu), so the offset and
 * the covariance become Q m and Q S Q^T. Exact: exp_{F mu}(Q nu) = F exp_mu(nu). */
void orc_rotate_component(const double F[9], const double mu[3], const double m[2], const double S[3],
                          double muw[3], double mw[2], double Sw[3])
{
    double R[9], Rw[9], Ft[6], Q[4];
    for (int i = 0; i < 3; ++i) muw[i] = F[3 * i] * mu[0] + F[3 * i + 1] * mu[1] + F[3 * i + 2] * mu[2];
    orc_frame(mu, R);
    orc_frame(muw, Rw);
    for (int j = 0; j < 2; ++j) /* F t_j(mu) */
        for (int i = 0; i < 3; ++i) Ft[3 * j + i] = F[3 * i] * R[3 * j] + F[3 * i + 1] * R[3 * j + 1] + F[3 * i + 2] * R[3 * j + 2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            Q[2 * i + j] = Rw[3 * i] * Ft[3 * j] + Rw[3 * i + 1] * Ft[3 * j + 1] + Rw[3 * i + 2] * Ft[3 * j + 2];
    mw[0] = Q[0] * m[0] + Q[1] * m[1];
    mw[1] = Q[2] * m[0] + Q[3] * m[1];
    double Sf[4] = {S[0], S[1], S[1], S[2]}, T[4];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) T[2 * i + j] = Q[2 * i] * Sf[j] + Q[2 * i + 1] * Sf[2 + j];
    Sw[0] = T[0] * Q[0] + T[1] * Q[1];
    Sw[1] = T[2] * Q[0] + T[3] * Q[1];
    Sw[2] = T[2] * Q[2] + T[3] * Q[3];
}

/* one pair of the product mixture, in the tangent space of the radiance component */
typedef struct {
    double logw;  /* log of pi'_k w_b N(m_k; a, A + B) (-inf for an empty pair) */
    double mu[3]; /* the radiance component's mean direction */
    double c[2];  /* product mean */
    double C[3];  /* product covariance, packed */
} orc_pair;

/* the two BSDF components of largest conditioned weight (lowest index on ties); sel[1]
 * is -1 when there is only one component or the second weight is zero */
static void top_two(int Kb, const double *w, int sel[2])
{
    sel[0] = sel[1] = -1;
    for (int b = 0; b < Kb; ++b) {
        if (!(w[b] > 0.0)) continue;
        if (sel[0] < 0 || w[b] > w[sel[0]]) {
            sel[1] = sel[0];
            sel[0] = b;
        } else if (sel[1] < 0 || w[b] > w[sel[1]]) {
            sel[1] = b;
        }
    }
}

/* Product of the conditioned radiance mixture of one query with its conditioned,
 * pruned and rotated BSDF mixture: pairs[2k + j] for radiance component k and the j-th
 * kept BSDF component. For each pair the BSDF component is moved into the tangent space
 * of mu_k (centre a, covariance B = J S_b J^T, orc_pair_transfer) and multiplied with
 * N(m_k, A = Sigma'_k): N(nu; m_k, A) N(nu; a, B) = N(m_k; a, A + B) N(nu; c, C) with
 * C = A (A + B)^-1 B and c = B (A + B)^-1 m_k + A (A + B)^-1 a. Returns -1 if a mixture
 * cannot be conditioned. */
int orc_product_pairs(int32_t K, const double *pi, const double *mud, const double *mux, const double *cov,
                      const double x[3], int32_t Kb, const double *bpi, const double *bmud, const double *bmux,
                      const double *bcov, const double bx[3], const double F[9], orc_pair *pairs)
{
    double pic[ORC_KMAX], m[2 * ORC_KMAX], Sc[3 * ORC_KMAX];
    double bpic[ORC_KMAX], bm[2 * ORC_KMAX], bSc[3 * ORC_KMAX];
    if (orc_condition(K, pi, mux, cov, x, pic, m, Sc)) return -1;
    if (orc_condition(Kb, bpi, bmux, bcov, bx, bpic, bm, bSc)) return -1;
    int sel[2];
    top_two(Kb, bpic, sel);
    for (int k = 0; k < K; ++k) {
        for (int j = 0; j < 2; ++j) {
            orc_pair *pr = pairs + 2 * k + j;
            pr->logw = -INFINITY;
            for (int i = 0; i < 3; ++i) pr->mu[i] = mud[3 * k + i];
            pr->c[0] = pr->c[1] = 0.0;
            pr->C[0] = pr->C[2] = 1.0;
            pr->C[1] = 0.0;
            const int b = sel[j];
            if (b < 0 || !(pic[k] > 0.0)) continue;
            double muw[3], mw[2], Sw[3], a[2], J[4];
            orc_rotate_component(F, bmud + 3 * b, bm + 2 * b, bSc + 3 * b, muw, mw, Sw);
            orc_pair_transfer(mud + 3 * k, muw, mw, a, J);
            /* B = J Sw J^T */
            double Sf[4] = {Sw[0], Sw[1], Sw[1], Sw[2]}, JS[4], B[4];
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c) JS[2 * r + c] = J[2 * r] * Sf[c] + J[2 * r + 1] * Sf[2 + c];
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c) B[2 * r + c] = JS[2 * r] * J[2 * c] + JS[2 * r + 1] * J[2 * c + 1];
            const double A[4] = {Sc[3 * k], Sc[3 * k + 1], Sc[3 * k + 1], Sc[3 * k + 2]};
            double S[4] = {A[0] + B[0], A[1] + B[1], A[2] + B[2], A[3] + B[3]};
            const double det = S[0] * S[3] - S[1] * S[2];
            if (!(det > 0.0)) continue;
            const double Si[4] = {S[3] / det, -S[1] / det, -S[2] / det, S[0] / det};
            const double d[2] = {m[2 * k] - a[0], m[2 * k + 1] - a[1]};
            const double q = d[0] * (Si[0] * d[0] + Si[1] * d[1]) + d[1] * (Si[2] * d[0] + Si[3] * d[1]);
            pr->logw = log(pic[k]) + log(bpic[b]) - 0.5 * q - 0.5 * log(det) - log(2.0 * ORC_PI);
            double ASi[4], BSi[4], C[4];
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c) {
                    ASi[2 * r + c] = A[2 * r] * Si[c] + A[2 * r + 1] * Si[2 + c];
                    BSi[2 * r + c] = B[2 * r] * Si[c] + B[2 * r + 1] * Si[2 + c];
                }
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c) C[2 * r + c] = ASi[2 * r] * B[c] + ASi[2 * r + 1] * B[2 + c];
            pr->C[0] = C[0];
            pr->C[1] = 0.5 * (C[1] + C[2]);
            pr->C[2] = C[3];
            for (int r = 0; r < 2; ++r)
                pr->c[r] = BSi[2 * r] * m[2 * k] + BSi[2 * r + 1] * m[2 * k + 1] + ASi[2 * r] * a[0] + ASi[2 * r + 1] * a[1];
        }
    }
    return 0;
}

/* normalised pair probabilities; 0 if every pair is empty */
static int pair_probs(int np, const orc_pair *pairs, double *P)
{
    double lmax = -INFINITY, den = 0.0;
    for (int p = 0; p < np; ++p)
        if (pairs[p].logw > lmax) lmax = pairs[p].logw;
    if (lmax == -INFINITY) return 0;
    for (int p = 0; p < np; ++p) den += exp(pairs[p].logw - lmax);
    for (int p = 0; p < np; ++p) P[p] = exp(pairs[p].logw - lmax) / den;
    return 1;
}

/* solid-angle density of the normalised product mixture at w: sum_p P_p N(log_{mu_p} w;
 * c_p, C_p) / sinc|log_{mu_p} w|, a pair contributing 0 at or beyond the cut locus */
static double product_density(int np, const orc_pair *pairs, const double *P, const double w[3])
{
    double pdf = 0.0;
    for (int p = 0; p < np; ++p) {
        if (!(P[p] > 0.0)) continue;
        double R[9], nu[2], L[3], d[2], z[2];
        orc_frame(pairs[p].mu, R);
        orc_log_map(R, w, nu);
        double r = hypot(nu[0], nu[1]);
        if (r >= ORC_PI * (1.0 - 1e-6)) continue;
        if (chol_packed(2, pairs[p].C, L) != 0) continue;
        d[0] = nu[0] - pairs[p].c[0];
        d[1] = nu[1] - pairs[p].c[1];
        forward_solve(2, L, d, z);
        double sinc = (r > 0.0) ? sin(r) / r : 1.0;
        pdf += P[p] * exp(-0.5 * (z[0] * z[0] + z[1] * z[1])) / (2.0 * ORC_PI * L[0] * L[2]) / sinc;
    }
    return pdf;
}

/* Product sampling for nq queries: radiance cell qcell[q] conditioned on qpos[q], BSDF
 * model bcell[q] conditioned on bpar[q], rotated by frames[9 q ...] (row-major F,
 * world = F local). Per draw (uniforms[(q ns + t) 3 + {0,1,2}] in [0,1)): the pair by the
 * CDF of the pair probabilities in order 2k + j (lowest index on ties), nu = c + chol(C) z
 * with z by Box-Muller (u1 mapped to (0,1]), discarded at |nu| >= pi, w = exp_{mu_k}(nu),
 * and the product density at w. Invalid draws give dir 0, pdf 0, valid 0, pair -1. */
int orc_product_sample(int32_t K, const double *pi, const double *mud, const double *mux, const double *cov,
                       int32_t Kb, const double *bpi, const double *bmud, const double *bmux, const double *bcov,
                       int64_t nq, const double *qpos, const int32_t *qcell, const double *bpar,
                       const int32_t *bcell, const double *frames, int32_t ns, const double *uniforms,
                       double *dirs_out, double *pdf_out, int32_t *pair_out, uint8_t *valid_out)
{
    orc_pair pairs[2 * ORC_KMAX];
    double P[2 * ORC_KMAX];
    for (int64_t q = 0; q < nq; ++q) {
        const int64_t ck = (int64_t)qcell[q] * K, cb = (int64_t)bcell[q] * Kb;
        if (orc_product_pairs(K, pi + ck, mud + 3 * ck, mux + 3 * ck, cov + 15 * ck, qpos + 3 * q, Kb, bpi + cb,
                              bmud + 3 * cb, bmux + 3 * cb, bcov + 15 * cb, bpar + 3 * q, frames + 9 * q, pairs))
            return -1;
        const int np = 2 * K;
        const int any = pair_probs(np, pairs, P);
        for (int t = 0; t < ns; ++t) {
            const double *u = uniforms + 3 * (q * ns + t);
            const int64_t o = q * ns + t;
            valid_out[o] = 0;
            pdf_out[o] = 0.0;
            pair_out[o] = -1;
            dirs_out[3 * o] = dirs_out[3 * o + 1] = dirs_out[3 * o + 2] = 0.0;
            if (!any) continue;
            int sel = -1;
            double cdf = 0.0;
            for (int p = 0; p < np; ++p) {
                cdf += P[p];
                if (u[0] < cdf) {
                    sel = p;
                    break;
                }
            }
            if (sel < 0)
                for (int p = np - 1; p >= 0; --p)
                    if (P[p] > 0.0) {
                        sel = p;
                        break;
                    }
            pair_out[o] = sel;
            double L[3];
            if (chol_packed(2, pairs[sel].C, L) != 0) continue;
            const double rad = sqrt(-2.0 * log(1.0 - u[1]));
            const double z0 = rad * cos(2.0 * ORC_PI * u[2]), z1 = rad * sin(2.0 * ORC_PI * u[2]);
            const double nu[2] = {pairs[sel].c[0] + L[0] * z0, pairs[sel].c[1] + L[1] * z0 + L[2] * z1};
            if (hypot(nu[0], nu[1]) >= ORC_PI) continue;
            double R[9], w[3];
            orc_frame(pairs[sel].mu, R);
            orc_exp_map(R, nu, w);
            valid_out[o] = 1;
            for (int d = 0; d < 3; ++d) dirs_out[3 * o + d] = w[d];
            pdf_out[o] = product_density(np, pairs, P, w);
        }
    }
    return 0;
}

/* the product density for nd given directions per query (dirs[(q nd + t) 3 ...]) */
int orc_product_pdf(int32_t K, const double *pi, const double *mud, const double *mux, const double *cov,
                    int32_t Kb, const double *bpi, const double *bmud, const double *bmux, const double *bcov,
                    int64_t nq, const double *qpos, const int32_t *qcell, const double *bpar, const int32_t *bcell,
                    const double *frames, int32_t nd, const double *dirs, double *pdf_out)
{
    orc_pair pairs[2 * ORC_KMAX];
    double P[2 * ORC_KMAX];
    for (int64_t q = 0; q < nq; ++q) {
        const int64_t ck = (int64_t)qcell[q] * K, cb = (int64_t)bcell[q] * Kb;
        if (orc_product_pairs(K, pi + ck, mud + 3 * ck, mux + 3 * ck, cov + 15 * ck, qpos + 3 * q, Kb, bpi + cb,
                              bmud + 3 * cb, bmux + 3 * cb, bcov + 15 * cb, bpar + 3 * q, frames + 9 * q, pairs))
            return -1;
        const int any = pair_probs(2 * K, pairs, P);
        for (int t = 0; t < nd; ++t)
            pdf_out[q * nd + t] = any ? product_density(2 * K, pairs, P, dirs + 3 * (q * nd + t)) : 0.0;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* spatial kD-tree: pre-subdivision, refinement, leaf initialisation          */
/* (Sec. 4.2 "Refinement of the spatial kD-tree"; Sec. 4.3 "Initialization")  */
/* ------------------------------------------------------------------------- */

/* Tree arrays (caller-owned): per node axis (0..2, -1 for a leaf), split position,
 * left child (the right child is left + 1) and leaf index (-1 for an inner node); per
 * leaf its node, its box and whether its mixture is initialised; counts[0] = nodes,
 * counts[1] = leaves. */
typedef struct {
    int32_t max_nodes, max_leaves;
    int32_t *counts;
    int32_t *axis, *left, *leaf;
    double *split;
    int32_t *leaf_node;
    double *lo, *hi; /* [max_leaves][3] */
    int32_t *init;
} orc_tree;

/* Pre-subdivision: `depth` rounds of splitting every leaf at the centre of x, then y,
 * then z, giving 8^depth equal boxes. Nodes in breadth-first order (children of node n
 * at 2n + 1, 2n + 2); leaves numbered left to right. No leaf is initialised. */
int orc_tree_init(orc_tree *t, int32_t depth, const double lo[3], const double hi[3])
{
    const int levels = 3 * depth;
    const int64_t n_leaves = (int64_t)1 << levels, n_nodes = 2 * n_leaves - 1;
    if (depth < 0 || n_nodes > t->max_nodes || n_leaves > t->max_leaves) return -1;
    double (*blo)[3] = malloc(sizeof(double[3]) * n_nodes), (*bhi)[3] = malloc(sizeof(double[3]) * n_nodes);
    for (int d = 0; d < 3; ++d) {
        blo[0][d] = lo[d];
        bhi[0][d] = hi[d];
    }
    for (int64_t n = 0; n < n_nodes; ++n) {
        int level = 0;
        while (((int64_t)1 << (level + 1)) - 1 <= n) ++level;
        if (level < levels) {
            const int ax = level % 3;
            const double mid = 0.5 * (blo[n][ax] + bhi[n][ax]);
            t->axis[n] = ax;
            t->split[n] = mid;
            t->left[n] = (int32_t)(2 * n + 1);
            t->leaf[n] = -1;
            for (int c = 0; c < 2; ++c) {
                const int64_t ch = 2 * n + 1 + c;
                for (int d = 0; d < 3; ++d) {
                    blo[ch][d] = blo[n][d];
                    bhi[ch][d] = bhi[n][d];
                }
                if (c == 0) bhi[ch][ax] = mid;
                else blo[ch][ax] = mid;
            }
        } else {
            const int64_t l = n - (n_leaves - 1);
            t->axis[n] = -1;
            t->split[n] = 0.0;
            t->left[n] = -1;
            t->leaf[n] = (int32_t)l;
            t->leaf_node[l] = (int32_t)n;
            for (int d = 0; d < 3; ++d) {
                t->lo[3 * l + d] = blo[n][d];
                t->hi[3 * l + d] = bhi[n][d];
            }
            t->init[l] = 0;
        }
    }
    t->counts[0] = (int32_t)n_nodes;
    t->counts[1] = (int32_t)n_leaves;
    free(blo);
    free(bhi);
    return 0;
}

/* the leaf containing position p: left where p[axis] < split, else right */
static int32_t tree_locate(const orc_tree *t, const double p[3])
{
    int32_t n = 0;
    while (t->axis[n] >= 0) n = (p[t->axis[n]] < t->split[n]) ? t->left[n] : t->left[n] + 1;
    return t->leaf[n];
}

/* The initial mixture of a leaf from its box (the recipe of the synthetic inputs, which
 * stands in for the k-means++ and surface-normal construction of the paper's App. B/C):
 * n_dir = min(8, K) directions at the cube vertices (+-1, +-1, +-1)/sqrt(3) in the order
 * x-sign, y-sign, z-sign (positive first), n_pos = ceil(K / n_dir) positions spread
 * along the longest box side (two: centre -+ d/4; four: a 2x2 pattern at -+d/4 on the two
 * longest sides; more: evenly at ((s + 1/2)/n_pos - 1/2) d), component k = s n_dir + v;
 * directional variance 2 pi / 8, positional variance r^2 / chi2_3^-1(0.9) with
 * r = 2 d / n_pos; weights 1/K. */
void orc_init_leaf(int32_t K, const double lo[3], const double hi[3], double *pi, double *mud, double *mux,
                   double *cov)
{
    const double chi2_3_inv_090 = 6.251388631170325;
    const int n_dir = K < 8 ? K : 8;
    const int n_pos = (K + n_dir - 1) / n_dir;
    double size[3], centre[3], d = 0.0;
    for (int a = 0; a < 3; ++a) {
        size[a] = hi[a] - lo[a];
        centre[a] = lo[a] + 0.5 * size[a];
        if (size[a] > d) d = size[a];
    }
    int order[3] = {0, 1, 2}; /* axes by decreasing size, stable */
    for (int i = 1; i < 3; ++i)
        for (int j = i; j > 0 && size[order[j]] > size[order[j - 1]]; --j) {
            int tmp = order[j];
            order[j] = order[j - 1];
            order[j - 1] = tmp;
        }
    const double r = 2.0 * d / n_pos;
    const double inv_sqrt3 = 1.0 / sqrt(3.0);
    for (int k = 0; k < K; ++k) {
        const int s = k / n_dir, v = k % n_dir;
        double off[3] = {0.0, 0.0, 0.0};
        if (n_pos == 2) {
            off[order[0]] = (s == 0 ? -1.0 : 1.0) * d / 4.0;
        } else if (n_pos == 4) {
            off[order[0]] = (s % 2 == 0 ? -1.0 : 1.0) * d / 4.0;
            off[order[1]] = (s / 2 == 0 ? -1.0 : 1.0) * d / 4.0;
        } else if (n_pos > 1) {
            off[order[0]] = ((s + 0.5) / n_pos - 0.5) * d;
        }
        for (int a = 0; a < 3; ++a) mux[3 * k + a] = centre[a] + off[a];
        mud[3 * k + 0] = ((v >> 2) & 1 ? -1.0 : 1.0) * inv_sqrt3;
        mud[3 * k + 1] = ((v >> 1) & 1 ? -1.0 : 1.0) * inv_sqrt3;
        mud[3 * k + 2] = (v & 1 ? -1.0 : 1.0) * inv_sqrt3;
        for (int q = 0; q < 15; ++q) cov[15 * k + q] = 0.0;
        cov[15 * k + TRI(0, 0)] = cov[15 * k + TRI(1, 1)] = 2.0 * ORC_PI / 8.0;
        for (int a = 0; a < 3; ++a) cov[15 * k + TRI(2 + a, 2 + a)] = r * r / chi2_3_inv_090;
        pi[k] = 1.0 / K;
    }
}

/* Refinement with the samples of one rendering iteration (positions in rows 3..5 of the
 * float32 [7][N] array), K-component mixtures and Robbins-Monro state per leaf:
 *   rounds: every leaf (first round) or every leaf created in the previous round (later
 *   rounds) with more than c samples is split along the axis of largest variance of its
 *   sample positions (ties: lowest axis), at their mean along that axis, if that leaves
 *   samples on both sides (some x < mean <= some other x); leaves split in increasing
 *   leaf order; the left child keeps the parent's leaf index and the right child takes
 *   the next new index; both get new nodes (left = the next free node); the parent's
 *   mixture, Robbins-Monro state and initialisation flag are copied to the right child.
 *   A split that would exceed the node or leaf capacity is not made (status bit 1).
 *   Rounds repeat until no leaf splits.
 *   Then every leaf with at least min_init samples whose mixture is not initialised gets
 *   the initial mixture of its box and a zero Robbins-Monro state.
 * Output: offsets[0..n_leaves] (samples per leaf, leaf order) and the samples reordered
 * by leaf, stably (index order within a leaf). Means and variances are FP64 sums over
 * the leaf's samples in index order. Returns the status bits, or -1 on bad arguments. */
int orc_tree_refine(orc_tree *t, const float *smp, int64_t N, int32_t c, int32_t min_init, int32_t K, double *pi,
                    double *mud, double *mux, double *cov, double *s0, double *s2, double *sw, int32_t *step,
                    float *sorted, int64_t *offsets)
{
    if (c < 1 || K < 1 || K > ORC_KMAX) return -1;
    int status = 0;
    int32_t *leaf_of = malloc(sizeof(int32_t) * (N > 0 ? N : 1));
    int32_t *active = malloc(sizeof(int32_t) * t->max_leaves);
    int32_t *next = malloc(sizeof(int32_t) * t->max_leaves);
    int64_t *cnt = malloc(sizeof(int64_t) * t->max_leaves);
    double *s1a = malloc(sizeof(double) * 3 * t->max_leaves), *sqa = malloc(sizeof(double) * 3 * t->max_leaves);
    double *mna = malloc(sizeof(double) * 3 * t->max_leaves), *mxa = malloc(sizeof(double) * 3 * t->max_leaves);
    int32_t n_active = t->counts[1];
    for (int32_t l = 0; l < n_active; ++l) active[l] = l;
    for (;;) {
        for (int64_t i = 0; i < N; ++i) {
            double p[3] = {smp[3 * N + i], smp[4 * N + i], smp[5 * N + i]};
            leaf_of[i] = tree_locate(t, p);
        }
        /* per-leaf count, sums, minima and maxima of the positions, in index order */
        const int32_t L0 = t->counts[1];
        for (int32_t l = 0; l < L0; ++l) {
            cnt[l] = 0;
            for (int d = 0; d < 3; ++d) {
                s1a[3 * l + d] = sqa[3 * l + d] = 0.0;
                mna[3 * l + d] = INFINITY;
                mxa[3 * l + d] = -INFINITY;
            }
        }
        for (int64_t i = 0; i < N; ++i) {
            const int32_t l = leaf_of[i];
            cnt[l] += 1;
            for (int d = 0; d < 3; ++d) {
                const double x = smp[(3 + d) * N + i];
                s1a[3 * l + d] += x;
                sqa[3 * l + d] += x * x;
                if (x < mna[3 * l + d]) mna[3 * l + d] = x;
                if (x > mxa[3 * l + d]) mxa[3 * l + d] = x;
            }
        }
        int32_t n_next = 0;
        for (int32_t a = 0; a < n_active; ++a) {
            const int32_t l = active[a];
            const int64_t M = cnt[l];
            const double *s1 = s1a + 3 * l, *sq = sqa + 3 * l, *mn = mna + 3 * l, *mx = mxa + 3 * l;
            if (M <= c) continue;
            int ax = 0;
            double best = -1.0, var[3];
            for (int d = 0; d < 3; ++d) {
                const double mean = s1[d] / (double)M;
                var[d] = sq[d] / (double)M - mean * mean;
                if (var[d] > best) {
                    best = var[d];
                    ax = d;
                }
            }
            const double split = s1[ax] / (double)M;
            if (!(mn[ax] < split && split <= mx[ax])) continue; /* not splittable */
            if (t->counts[0] + 2 > t->max_nodes || t->counts[1] + 1 > t->max_leaves) {
                status |= 1;
                continue;
            }
            const int32_t n = t->leaf_node[l];
            const int32_t L = t->counts[0], r = t->counts[1];
            t->axis[n] = ax;
            t->split[n] = split;
            t->left[n] = L;
            t->leaf[n] = -1;
            t->axis[L] = t->axis[L + 1] = -1;
            t->left[L] = t->left[L + 1] = -1;
            t->split[L] = t->split[L + 1] = 0.0;
            t->leaf[L] = l;
            t->leaf[L + 1] = r;
            t->leaf_node[l] = L;
            t->leaf_node[r] = L + 1;
            for (int d = 0; d < 3; ++d) {
                t->lo[3 * r + d] = t->lo[3 * l + d];
                t->hi[3 * r + d] = t->hi[3 * l + d];
            }
            t->hi[3 * l + ax] = split;
            t->lo[3 * r + ax] = split;
            t->init[r] = t->init[l];
            memcpy(pi + (int64_t)r * K, pi + (int64_t)l * K, sizeof(double) * K);
            memcpy(mud + (int64_t)r * K * 3, mud + (int64_t)l * K * 3, sizeof(double) * 3 * K);
            memcpy(mux + (int64_t)r * K * 3, mux + (int64_t)l * K * 3, sizeof(double) * 3 * K);
            memcpy(cov + (int64_t)r * K * 15, cov + (int64_t)l * K * 15, sizeof(double) * 15 * K);
            memcpy(s0 + (int64_t)r * K, s0 + (int64_t)l * K, sizeof(double) * K);
            memcpy(s2 + (int64_t)r * K * 15, s2 + (int64_t)l * K * 15, sizeof(double) * 15 * K);
            sw[r] = sw[l];
            step[r] = step[l];
            t->counts[0] += 2;
            t->counts[1] += 1;
            next[n_next++] = l;
            next[n_next++] = r;
        }
        if (n_next == 0) break;
        /* the next round looks at the children, in increasing leaf order */
        for (int32_t i = 1; i < n_next; ++i)
            for (int32_t j = i; j > 0 && next[j] < next[j - 1]; --j) {
                int32_t tmp = next[j];
                next[j] = next[j - 1];
                next[j - 1] = tmp;
            }
        memcpy(active, next, sizeof(int32_t) * n_next);
        n_active = n_next;
    }
    /* counts, offsets and the stable reordering */
    const int32_t L = t->counts[1];
    for (int32_t l = 0; l <= L; ++l) offsets[l] = 0;
    for (int64_t i = 0; i < N; ++i) offsets[leaf_of[i] + 1] += 1;
    for (int32_t l = 0; l < L; ++l) offsets[l + 1] += offsets[l];
    int64_t *fill = malloc(sizeof(int64_t) * (L > 0 ? L : 1));
    for (int32_t l = 0; l < L; ++l) fill[l] = offsets[l];
    for (int64_t i = 0; i < N; ++i) {
        const int64_t o = fill[leaf_of[i]]++;
        for (int a = 0; a < 7; ++a) sorted[(int64_t)a * N + o] = smp[(int64_t)a * N + i];
    }
    /* initialisation of leaves that reached min_init samples */
    for (int32_t l = 0; l < L; ++l) {
        if (t->init[l] || offsets[l + 1] - offsets[l] < min_init) continue;
        const int64_t g = (int64_t)l * K;
        orc_init_leaf(K, t->lo + 3 * l, t->hi + 3 * l, pi + g, mud + 3 * g, mux + 3 * g, cov + 15 * g);
        memset(s0 + g, 0, sizeof(double) * K);
        memset(s2 + 15 * g, 0, sizeof(double) * 15 * K);
        sw[l] = 0.0;
        step[l] = 0;
        t->init[l] = 1;
    }
    free(fill);
    free(leaf_of);
    free(active);
    free(next);
    free(cnt);
    free(s1a);
    free(sqa);
    free(mna);
    free(mxa);
    return status;
}

/* ------------------------------------------------------------------------- */
/* counter-based uniforms: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)  */
/* ------------------------------------------------------------------------- */

/* ten rounds of the Philox S-P network on a 4x32-bit counter with a 2x32-bit key */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* the library's uniforms for draw d under seed s: counter (d_lo, d_hi, 0, 0), key
 * (s_lo, s_hi); the first three outputs give (x >> 8) * 2^-24 in [0, 1) */
void orc_draw_uniforms(uint64_t seed, int64_t n, double *u /* [n][3] */)
{
    for (int64_t d = 0; d < n; ++d) {
        uint32_t c[4] = {(uint32_t)d, (uint32_t)((uint64_t)d >> 32), 0u, 0u};
        uint32_t k[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
        uint32_t o[4];
        orc_philox4x32_10(c, k, o);
        for (int j = 0; j < 3; ++j) u[3 * d + j] = (double)(o[j] >> 8) * (1.0 / 16777216.0);
    }
}

/* Threads of the OpenMP build (the all-cores CPU baseline); returns the count in use.
 * The single-threaded build ignores the request and returns 1. */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
