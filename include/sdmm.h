/*
 * sdmm.h -- C ABI of libsdmm, an MI355X (gfx950) implementation of the data-parallel
 * core of "Path Guiding Using Spatio-Directional Mixture Models" (Dodik, Papas,
 * Oztireli, Mueller; arXiv 2111.13094):
 *
 *   - weighted MAP EM with Robbins-Monro averaging for many independent K-component
 *     Gaussian mixtures over direction x position, directions taken in each component's
 *     tangent space (Sec. 3.1-3.4, Sec. 4.2-4.3 of the paper);
 *   - closed-form conditioning of a fitted 5-D mixture on a position, the solid-angle
 *     pdf of the conditioned directional mixture, and sampling from it (Sec. 3.1-3.3);
 *   - the gradient of the weighted penalised log-likelihood (adjoint).
 *
 * Conventions for every entry point
 *   - Pointers marked [device] are device memory on the current HIP device; [host] are
 *     host memory. All buffers are owned by the caller; the library keeps no model state.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream. Every call
 *     only enqueues work on that stream and returns without synchronising, except where
 *     stated. Results are valid once the stream has been synchronised.
 *   - Return value: SDMM_OK or a negative SDMM_E* code. Nothing is enqueued when a call
 *     returns an error. Numerical conditions are not errors: they are reported per cell
 *     in `cell_status` (SDMM_CELL_* bits) and leave that cell's parameters and state
 *     untouched (SKIPPED_*, BAD_*).
 *   - Samples: float32 structure-of-arrays [7][n_samples] = dir x, y, z (unit vectors),
 *     pos x, y, z (normalised to the unit cube, Sec. 4.3), Monte Carlo weight >= 0.
 *     Cell c owns samples [cell_offsets[c], cell_offsets[c+1]) (int64, non-decreasing).
 *   - Mixtures: float64 masters, component index fastest within a cell:
 *     weights [n_cells*K], mean_dir [n_cells*K*3] (unit), mean_pos [n_cells*K*3],
 *     cov [n_cells*K*15] = 5x5 SPD covariance, packed lower triangle row-major
 *     (index d(d+1)/2+e, d>=e) in the coordinate order (nu_u, nu_v, x, y, z); nu is the
 *     tangent coordinate of the direction in the frame R_mu whose rows are (t1, t2, mu),
 *     t1 and t2 from the branchless orthonormal basis of Duff et al. (2017).
 */
#ifndef SDMM_H
#define SDMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define SDMM_OK 0
#define SDMM_EINVAL (-1)       /* bad argument: null pointer, size, K out of range, ... */
#define SDMM_EDEVICE (-2)      /* a HIP runtime call failed */
#define SDMM_ENOWORKSPACE (-3) /* workspace smaller than the *_workspace_size() value */

/* ---- per-cell status bits (OR over the iterations of one call) ---- */
#define SDMM_CELL_SKIPPED_FEW 1    /* fewer than min_samples positive weights (Sec. 4.2) */
#define SDMM_CELL_SKIPPED_ZERO_W 2 /* the weights sum to zero */
#define SDMM_CELL_BAD_INPUT 4      /* negative weight, or non-finite sample / statistic */
#define SDMM_CELL_DEAD_COMPONENT 8 /* some component kept its mean and covariance because
                                      its normalised weight sum was <= dead_threshold */
#define SDMM_CELL_CHOL_FAIL_KEPT_PREV 16 /* some updated covariance was not SPD; the previous
                                            one was kept */
#define SDMM_CELL_BAD_PARAMS 32    /* input mixture not usable: non-finite or negative
                                      weight, non-finite mean, non-SPD covariance */

/* ---- options ---- */
#define SDMM_ETA_CONSTANT 0 /* eta_j = 1 for j = 0, eta for j > 0 */
#define SDMM_ETA_PAPER 1    /* eta_j = (rm_beta * j + 1)^(-rm_alpha) (Sec. 4.3) */
#define SDMM_PRIOR_ETA_OVER_M 0 /* prior strength beta_j = eta_j / M_j, M_j = #{w > 0} */
#define SDMM_PRIOR_FIXED 1      /* beta_j = prior_scale */

#define SDMM_FLAG_ESTEP_JACOBIAN 1 /* responsibilities from solid-angle densities instead of
                                      the tangent densities of the statistics equation */
#define SDMM_FLAG_PLAIN_FP32 2     /* precision study: plain FP32 running sums */
#define SDMM_FLAG_FP64_SUMS 4      /* precision study: FP64 running sums */
#define SDMM_FLAG_ACCURATE_SIGMA 8 /* accurate covariance update (Sec. 3.2, statistics in the
                                      new mean's tangent space): after the M-step has moved
                                      the weights and means, a second E-step pass under
                                      (new weights, new means, previous covariances) forms
                                      S0' = sum w r' and S2' = sum w r' y^ y^^T with y^ the
                                      coordinates about the new mean, and
                                      Sigma = (beta B + S2' / W) / (beta a + S0' / W).
                                      Batch steps only: needs eta_mode SDMM_ETA_CONSTANT with
                                      eta = 1 and the batched or per-cell schedule (else
                                      SDMM_EINVAL). Twice the E-step work. */
#define SDMM_FLAG_CARRY_MIRRORS 16 /* batched schedule, for callers whose mixtures change
                                      only through these calls (a fitting loop over
                                      successive batches): the last M-step also writes the
                                      FP32 E-step mirrors of the new parameters into the
                                      workspace, and a call with this flag whose workspace's
                                      previous call did so for the same mixture arrays
                                      (pointers, n_cells, K) skips the setup kernel that
                                      would rebuild them: its E-step launch checks the
                                      offsets and its M-step resets the statuses. The
                                      library keeps that record on the host; any other call
                                      on the workspace (another schedule, no flag, a failed
                                      call, sdmm_fit_grad) clears it. Results are bit for
                                      bit those without the flag. Changing the mixture
                                      values between two flagged calls on one workspace
                                      (other than through these calls) leaves stale mirrors:
                                      clear the flag for the next call. Ignored by the other
                                      schedules. */

#define SDMM_SCHED_BATCHED 0  /* per iteration one E launch for all cells, then one M
                                 launch for all cells */
#define SDMM_SCHED_PER_CELL 1 /* plain baseline: one E and one M launch per cell; copies
                                 cell_offsets to the host and synchronises the stream */
#define SDMM_SCHED_FUSED 2    /* one E+M launch per iteration: the last wave to finish a
                                 cell's E-step items runs that cell's M-step */
#define SDMM_SCHED_STEPWISE 3 /* stepwise EM (Sec. 6, "Mini-batch EM versus stepwise EM"):
                                 each sample with positive weight, in index order, is a
                                 mini-batch of one (blend with eta_j for the cell's sample
                                 counter j, MAP M-step with M = 1, transport of the carried
                                 S2); a fresh cell (step 0) first takes one batch step over
                                 its samples. One wave per cell, FP64 throughout (the
                                 precision flags have no effect); iters passes. */

typedef struct sdmm_fit_opts {
    int32_t K;           /* components per cell, 1..64 */
    int32_t iters;       /* E+M iterations over the given batch, >= 1 */
    int32_t eta_mode;    /* SDMM_ETA_* */
    int32_t prior_mode;  /* SDMM_PRIOR_* */
    int32_t flags;       /* SDMM_FLAG_* */
    int32_t min_samples; /* 16 in the paper (Sec. 4.2) */
    int32_t schedule;    /* SDMM_SCHED_* */
    int32_t min_range;   /* E-step work split: the samples are cut into ranges of
                            P = max(min_range, ceil(N / max_ranges)) samples and each
                            (cell, range) intersection is one wave's work item;
                            0 = 256. Results do not depend on it beyond FP rounding. */
    int32_t max_ranges;  /* upper bound on the number of ranges, 0 = 65536, at most 2^20 */
    int32_t use_graph;   /* 1: capture the iteration sequence in a hipGraph, cached by
                            argument values, and replay it */
    int32_t waves_per_block; /* E-step launch: 1, 2 or 4 waves (work items) per work
                            group; 0 = 1. Single-wave groups let a compute unit start a
                            new item as soon as any wave slot frees up. */
    int32_t max_cell_samples; /* hint: no cell of the batch holds more samples than this
                            (for cells that are kD-tree leaves, the split threshold);
                            0 = no bound, negative is rejected. It only bounds how many
                            record-tree levels are launched (each a kernel launch): a cell
                            above it is still fitted, its M-step then sums more records,
                            in a different order (FP64 rounding). */
    double eta;          /* Robbins-Monro weight of a new batch for SDMM_ETA_CONSTANT */
    double rm_alpha, rm_beta; /* SDMM_ETA_PAPER schedule (paper: 0.5, 0.1) */
    double prior_scale;  /* beta for SDMM_PRIOR_FIXED */
    double prior_q;      /* Dirichlet parameter (paper: 1/K) */
    double prior_a;      /* inverse-Wishart denominator (paper: 5/K) */
    double prior_b[5];   /* diagonal of B (paper: a * (0.1, 0.1, 1, 1, 1) * 1e-4) */
    double dead_threshold; /* normalised weight sum at or below which a component is dead */
} sdmm_fit_opts;

typedef struct sdmm_mixtures {
    int32_t n_cells;
    int32_t K;
    double *weights;  /* [device] n_cells*K */
    double *mean_dir; /* [device] n_cells*K*3 */
    double *mean_pos; /* [device] n_cells*K*3 */
    double *cov;      /* [device] n_cells*K*15 */
} sdmm_mixtures;

/* Robbins-Monro state (Sec. 4.3): averaged statistics carried into the frame of the
 * current means (first moment zero), averaged normaliser, and the per-cell step j.
 * Zero-initialised state (step 0) starts a fresh fit. */
typedef struct sdmm_em_state {
    double *s0;    /* [device] n_cells*K */
    double *s2;    /* [device] n_cells*K*15 (packed like cov) */
    double *sw;    /* [device] n_cells */
    int32_t *step; /* [device] n_cells */
} sdmm_em_state;

/* Bytes of device workspace sdmm_fit_mixtures needs for these sizes and options. */
size_t sdmm_fit_workspace_size(int32_t n_cells, int32_t K, int64_t n_samples,
                               const sdmm_fit_opts *opts);

/*
 * sdmm_fit_mixtures -- opts->iters iterations of weighted MAP EM on every cell.
 *
 * Per cell and iteration (paper Sec. 3.2, 3.4, 4.2, 4.3):
 *   gate: skip with a status bit unless M = #{w > 0} >= min_samples and sum w > 0;
 *   E-step: y_ik = (log_{mu_k}(w_i), p_i - mu_x_k); responsibilities r_ik from the
 *     tangent densities pi_k N5(y_ik; 0, Sigma_k); S0 = sum w r, S1 = sum w r y,
 *     S2 = sum w r y y^T, W = sum w (FP32 products, compensated FP32 running sums,
 *     FP64 reductions across lanes and work items);
 *   Robbins-Monro: S^ = (1 - eta_j) S^_prev + eta_j S (first batch: S^ = S), same for W;
 *   M-step (FP64): m = S1^/S0^; mu_dir <- exp_{mu_dir}(m_nu), mu_pos += m_x;
 *     C = S2^ - S1^ S1^T / S0^ moved to the new mean's frame by T = blkdiag(J, I3), J the
 *     Jacobian of log_{mu_new} o exp_{mu} at m; Sigma = (beta_j B + T C T^T / W^) /
 *     (beta_j a + S0^ / W^); pi = (beta_j q + S0^/W^) / (K beta_j q + sum S0^/W^);
 *     the carried state becomes S0^ and T C T^T; step += 1.
 *   With SDMM_FLAG_ACCURATE_SIGMA the covariance instead comes from the second pass
 *     described at the flag, and the carried S0 and S2 are S0' and S2'. Other flag bits
 *     are rejected.
 *
 * cell_offsets [device] int64[n_cells+1]; samples [device] float32[7][n_samples];
 * mix, state: device arrays updated in place; opts [host]; cell_status [device]
 * int32[n_cells] (overwritten); workspace [device] of at least
 * sdmm_fit_workspace_size() bytes (contents need not be initialised; not retained
 * between calls). Fitting cells together gives bitwise the same result as fitting each
 * cell alone, and repeated calls are bitwise reproducible (fixed reduction order).
 */
int sdmm_fit_mixtures(const int64_t *cell_offsets, const float *samples, int64_t n_samples,
                      const sdmm_mixtures *mix, const sdmm_em_state *state,
                      const sdmm_fit_opts *opts, int32_t *cell_status, void *workspace,
                      size_t workspace_bytes, void *stream);

/* Size of the library's own device workspace for sdmm_fit_mixtures_noalloc: 64 MiB per
 * device, held from the library's load to the end of the process. */
#define SDMM_NOALLOC_SCRATCH_BYTES (64u << 20)

/*
 * sdmm_fit_mixtures_noalloc -- sdmm_fit_mixtures for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc. Same arguments, kernels and results as sdmm_fit_mixtures (bitwise),
 * without the workspace: the library's static per-device array of
 * SDMM_NOALLOC_SCRATCH_BYTES takes its place. The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine); the first call on a device looks up that
 * device's array address once.
 * Limits: sdmm_fit_workspace_size() of the call must be at most
 * SDMM_NOALLOC_SCRATCH_BYTES, else SDMM_ENOWORKSPACE and nothing is enqueued (the
 * 4096-cell, 4.2M-sample batch fits with 512-sample work items, opts->min_range = 512);
 * opts->schedule SDMM_SCHED_PER_CELL and opts->use_graph = 1 are rejected with
 * SDMM_EINVAL (the first copies the offsets to the host, the second instantiates
 * graphs). Every call on a device shares that device's array: calls that overlap on
 * one device (different streams, or threads) race and must be serialised by the caller.
 * Nothing in the array needs to start at zero: each call resets what it reads.
 */
int sdmm_fit_mixtures_noalloc(const int64_t *cell_offsets, const float *samples, int64_t n_samples,
                              const sdmm_mixtures *mix, const sdmm_em_state *state,
                              const sdmm_fit_opts *opts, int32_t *cell_status, void *stream);

/* ---- conditioning, pdf, sampling ---- */

/* floats per component in the conditioning table */
#define SDMM_COND_TABLE_STRIDE 32

/*
 * sdmm_condition_prepare -- the query-independent part of conditioning on the position
 * (paper Sec. 3.2 first paragraph, Sec. 3.3), per component, in FP64 and stored FP32:
 * the frame R_mu, mu_x, the Cholesky factor of Sigma_xx (inverted), the regression
 * A = Sigma_nx Sigma_xx^-1, the Cholesky factor L' of the conditional covariance
 * Sigma' = Sigma_nn - A Sigma_xn (and its inverse), and the log normalisers.
 * table [device] float32[n_cells*K*SDMM_COND_TABLE_STRIDE], written; the order of the
 * entries inside it is the library's own (only the size is part of the interface).
 */
int sdmm_condition_prepare(const sdmm_mixtures *mix, float *table, void *stream);

/*
 * sdmm_condition -- per query q (position qpos, cell qcell[q]):
 *   pi'_k = pi_k N3(x - mu_x_k; 0, Sigma_xx,k) / sum_j (...),  m_k = A_k (x - mu_x_k).
 * qpos [device] float32[3][nq] (SoA); qcell [device] int32[nq] in [0, n_cells);
 * cond_w [device] float32[nq][K]; cond_m [device] float32[nq][K][2] (written).
 */
int sdmm_condition(const float *table, int32_t n_cells, int32_t K, const float *qpos,
                   const int32_t *qcell, int64_t nq, float *cond_w, float *cond_m, void *stream);

/*
 * sdmm_pdf -- solid-angle pdf of the conditioned mixture (paper Sec. 3.1, mixture pdf):
 *   p(w | x) = sum_k pi'_k N2(nu_k - m_k; 0, Sigma'_k) / sinc|nu_k|, nu_k = log_{mu_k}(w),
 *   a component contributing 0 where |nu_k| >= pi (1 - 1e-6) (cut locus).
 * nd directions per query: dirs [device] float32[3][nq*nd] (SoA, direction t of query q
 * at column q*nd+t); pdf_out [device] float32[nq*nd].
 */
int sdmm_pdf(const float *table, int32_t n_cells, int32_t K, const int32_t *qcell, int64_t nq,
             const float *cond_w, const float *cond_m, int32_t nd, const float *dirs,
             float *pdf_out, void *stream);

/*
 * sdmm_sample -- ns draws per query (paper Sec. 3.1, "Sampling"): component by the CDF
 * of pi' (lowest index on ties), nu = m_k + L'_k z with z by Box-Muller from (u1, u2)
 * (u1 mapped to (0, 1] as 1 - u1), discarded when |nu| >= pi; w = exp_{mu_k}(nu); and
 * p(w | x) of the whole conditioned mixture.
 * uniforms [device] float32[3][nq*ns] in [0,1) (u0 picks the component) or NULL for
 * the device generator: Philox4x32-10 keyed by seed, counter (draw index, 0, 0, 0).
 * dirs_out [device] float32[3][nq*ns]; pdf_out [device] float32[nq*ns];
 * valid_out [device] uint8[nq*ns]; comp_out [device] int32[nq*ns] or NULL.
 * Discarded draws: valid 0, direction (0,0,0), pdf 0.
 */
int sdmm_sample(const float *table, int32_t n_cells, int32_t K, const int32_t *qcell, int64_t nq,
                const float *cond_w, const float *cond_m, int32_t ns, const float *uniforms,
                uint64_t seed, float *dirs_out, float *pdf_out, uint8_t *valid_out,
                int32_t *comp_out, void *stream);

/*
 * sdmm_condition_sample_pdf -- conditioning, sampling and pdf in one pass per query
 * without materialising pi' and m (same results as sdmm_condition + sdmm_sample).
 */
int sdmm_condition_sample_pdf(const float *table, int32_t n_cells, int32_t K, const float *qpos,
                              const int32_t *qcell, int64_t nq, int32_t ns, const float *uniforms,
                              uint64_t seed, float *dirs_out, float *pdf_out, uint8_t *valid_out,
                              void *stream);

/* ---- spatial kD-tree (Sec. 4.2 "Refinement of the spatial kD-tree"; Sec. 4.3
 *      "Initialization") ---- */

/* A kD-tree over positions whose leaves are the cells of the mixtures. Nodes: split axis
 * (0..2) and position (a point with p[axis] < split goes left), left child (the right
 * child is left + 1), and for a leaf node its leaf index. Leaves: their node, box and
 * whether their mixture is initialised. All arrays [device], caller-owned; counts[0] is
 * the number of nodes in use, counts[1] the number of leaves. */
typedef struct sdmm_tree {
    int32_t max_nodes;  /* capacity, at least 2 max_leaves - 1 */
    int32_t max_leaves; /* capacity: the cells of the mixtures and state */
    int32_t *counts;    /* int32[2] */
    int32_t *axis;      /* int32[max_nodes]: split axis, -1 for a leaf */
    int32_t *left;      /* int32[max_nodes]: left child, -1 for a leaf */
    int32_t *leaf;      /* int32[max_nodes]: leaf index of a leaf node, -1 otherwise */
    double *split;      /* float64[max_nodes]: split position */
    int32_t *leaf_node; /* int32[max_leaves]: the node of each leaf */
    double *lo, *hi;    /* float64[max_leaves][3]: leaf boxes */
    int32_t *init;      /* int32[max_leaves]: 1 once the leaf's mixture is initialised */
} sdmm_tree;

/*
 * sdmm_tree_init -- the pre-subdivision of Sec. 4.3: `depth` rounds (0..6) of splitting
 * every leaf at the centre of x, then y, then z, giving 8^depth equal boxes of the box
 * [lo, hi) (lo, hi [host] float64[3], lo < hi). Nodes are numbered breadth first
 * (children of node n at 2n + 1 and 2n + 2), leaves left to right; no leaf is
 * initialised. SDMM_EINVAL if the capacity is too small.
 */
int sdmm_tree_init(const sdmm_tree *tree, int32_t depth, const double *lo, const double *hi, void *stream);

/* Bytes of device workspace sdmm_tree_refine needs. */
size_t sdmm_tree_workspace_size(int64_t n_samples, int32_t max_leaves);

/*
 * sdmm_tree_refine -- adapts the tree to one iteration's samples and reorders them by
 * leaf for sdmm_fit_mixtures (Sec. 4.2, 4.3):
 *   rounds: every leaf (first round) or every leaf made in the previous round that holds
 *   more than split_threshold samples (the paper's c = 16000) is split at the mean of its
 *   sample positions along the axis of largest variance (lowest axis on ties), provided
 *   samples fall on both sides; leaves split in increasing leaf order, the left child
 *   keeping the parent's leaf index, the right child taking the next one; the new leaf
 *   gets a copy of the parent's mixture, Robbins-Monro state and initialisation flag.
 *   Splits beyond the node or leaf capacity are skipped (status bit 1). Rounds repeat
 *   until none splits (at most 64).
 *   Then every leaf with at least min_init samples (the paper's 16) whose mixture is not
 *   initialised gets the initial mixture of its box: min(8, K) directions at the cube
 *   vertices crossed with ceil(K / 8) positions along the longest sides, directional
 *   variance 2 pi / 8, positional variance (2 d / n_pos)^2 / chi2_3^-1(0.9) with d the
 *   longest side, weights 1/K; its Robbins-Monro state is zeroed.
 * samples [device] float32[7][n_samples] (as sdmm_fit_mixtures; n_samples < 2^31);
 * mix, state: [device] arrays for tree->max_leaves cells (mix->n_cells must equal it),
 * updated in place; sorted_out [device] float32[7][n_samples]: the samples by leaf, in
 * index order within a leaf; cell_offsets_out [device] int64[max_leaves + 1], of which
 * the first n_leaves + 1 entries are written; n_leaves_out, status_out [host] int32
 * (status_out may be NULL). The call synchronises the stream once per round. Means and
 * variances are FP64 sums over each leaf's samples. SDMM_EINVAL for bad arguments, or
 * when the tree's counts (read from the device) are out of range, in which case only the
 * workspace has been written. The call keeps one pinned 16-byte host buffer per host
 * thread for the counts it reads back.
 */
int sdmm_tree_refine(const sdmm_tree *tree, const float *samples, int64_t n_samples, int32_t split_threshold,
                     int32_t min_init, const sdmm_mixtures *mix, const sdmm_em_state *state,
                     float *sorted_out, int64_t *cell_offsets_out, int32_t *n_leaves_out,
                     int32_t *status_out, void *workspace, size_t workspace_bytes, void *stream);

/* ---- product sampling with a conditioned BSDF mixture ---- */

/*
 * sdmm_product_sample -- ns draws per query from the product of the conditioned radiance
 * mixture and a conditioned BSDF mixture (paper Sec. 3.4; pruning of Sec. 4.1).
 * Per query q:
 *   radiance: cell qcell[q] of `table` (sdmm_condition_prepare of the radiance mixtures,
 *     n_cells x K) conditioned on qpos[q] as in sdmm_condition: pi'_k, m_k, Sigma'_k in
 *     the tangent space of mu_k;
 *   BSDF: model bcell[q] of `btable` (sdmm_condition_prepare of BSDF models: 5-D
 *     mixtures over (local incident direction; three BSDF inputs such as the outgoing
 *     polar angle, azimuth and roughness), n_bsdf x Kb) conditioned on bpar[q]; the two
 *     components of largest conditioned weight are kept (lowest index on ties);
 *   each kept BSDF component is rotated to world by the shading frame F (world = F local):
 *     mean F mu_b, offset and covariance carried into the frame of F mu_b exactly;
 *   pair (k, j), radiance component k and the j-th kept BSDF component: the BSDF
 *     component in the tangent space of mu_k, centre a = log_{mu_k}(exp_{mu_b}(m_b)) and
 *     covariance J Sigma'_b J^T with J the Jacobian of log_{mu_k} o exp_{mu_b} at m_b; the
 *     product N(m_k, Sigma'_k) N(a, J Sigma'_b J^T) = lambda N(c, C) with
 *     lambda = pi'_k w_b N(m_k; a, Sigma'_k + J Sigma'_b J^T);
 *   draw: pair by the CDF of the normalised lambda in the order 2k + j (lowest index on
 *     ties), nu = c + chol(C) z with z by Box-Muller from (u1, u2) (u1 mapped to (0, 1] as
 *     1 - u1), discarded when |nu| >= pi, w = exp_{mu_k}(nu); and the solid-angle density
 *     of the normalised product mixture at w (sum of P N(log_{mu_k} w; c, C) /
 *     sinc|log_{mu_k} w|, a pair contributing 0 at |nu| >= pi (1 - 1e-6)).
 * qpos, bpar [device] float32[3][nq] (SoA); qcell [device] int32[nq] in [0, n_cells);
 * bcell [device] int32[nq] in [0, n_bsdf); frames [device] float32[9][nq] (SoA, entry
 * (r, c) of F at row 3r + c); uniforms [device] float32[3][nq*ns] in [0, 1) or NULL for
 * the device generator (as sdmm_sample). dirs_out [device] float32[3][nq*ns] (world);
 * pdf_out [device] float32[nq*ns]; valid_out [device] uint8[nq*ns]; pair_out [device]
 * int32[nq*ns] (2k + j, or -1) or NULL. A query whose cell or model index is out of range,
 * or whose pairs are all empty, and every discarded draw, give valid 0, direction
 * (0, 0, 0), pdf 0. K and Kb in 1..64; SDMM_EINVAL otherwise.
 */
int sdmm_product_sample(const float *table, int32_t n_cells, int32_t K, const float *qpos,
                        const int32_t *qcell, const float *btable, int32_t n_bsdf, int32_t Kb,
                        const float *bpar, const int32_t *bcell, const float *frames, int64_t nq,
                        int32_t ns, const float *uniforms, uint64_t seed, float *dirs_out,
                        float *pdf_out, uint8_t *valid_out, int32_t *pair_out, void *stream);

/*
 * sdmm_product_pdf -- the density of the normalised product mixture of
 * sdmm_product_sample at nd given world directions per query (dirs [device]
 * float32[3][nq*nd], direction t of query q at column q*nd+t; pdf_out [device]
 * float32[nq*nd]); 0 for a query without pairs.
 */
int sdmm_product_pdf(const float *table, int32_t n_cells, int32_t K, const float *qpos,
                     const int32_t *qcell, const float *btable, int32_t n_bsdf, int32_t Kb,
                     const float *bpar, const int32_t *bcell, const float *frames, int64_t nq,
                     int32_t nd, const float *dirs, float *pdf_out, void *stream);

/* ---- adjoint ---- */

/*
 * sdmm_fit_grad -- value and gradient of the weighted penalised log-likelihood
 *   F = sum_i (w_i / W) log sum_k pi_k N5(y_ik; 0, Sigma_k)
 *       + sum_k [beta q log pi_k - (beta a / 2) log det Sigma_k - (beta / 2) tr(B Sigma_k^-1)]
 * (the objective whose maximiser is the MAP update of Sec. 4.3) per cell, at the current
 * mixture, with beta = opts->prior_scale (and q, a, B from opts). Gradients are with
 * respect to the weight logits (pi = softmax), the positional means, a tangent
 * perturbation delta of each directional mean (mu(delta) = exp_mu(delta), frame rebuilt
 * at mu(delta)), and the packed Cholesky factor L of Sigma.
 * F_out [device] float64[n_cells]; g_alpha [device] float64[n_cells*K];
 * g_mu_pos, g_delta [device] float64[n_cells*K*3], [n_cells*K*2];
 * g_L [device] float64[n_cells*K*15]; cell_status [device] int32[n_cells] (gate as in
 * sdmm_fit_mixtures with min_samples; skipped cells get F = 0 and zero gradients).
 * workspace: at least sdmm_fit_workspace_size(n_cells, K, n_samples, opts) bytes.
 * Precision: by default the pass forms tangent coordinates and products in FP32 with
 * compensated sums and the quadratic form in FP64. Its relative rounding of 2^-24 in the
 * tangent coordinates is amplified by Sigma^-1 in the mean and factor gradients, by about
 * the condition number kappa of the component's correlation matrix: they agree with the
 * closed form to about 1e-4 of their scale where kappa <= 1e5, and resolve a fixed point
 * of EM (gradient below 2e-3 of its early size) only where kappa <= 1e3. With
 * SDMM_FLAG_FP64_SUMS in opts->flags every per-sample quantity is FP64 (verification
 * mode: about 3x slower; its parameters enter as hi/lo FP32 pairs, about 48 bits),
 * agreeing with the closed form to about 1e-7 on every component; use it for
 * stationarity checks of converged, strongly correlated components.
 * SDMM_FLAG_ESTEP_JACOBIAN is rejected (SDMM_EINVAL); SDMM_FLAG_ACCURATE_SIGMA, an
 * M-step option, has no effect here.
 */
int sdmm_fit_grad(const int64_t *cell_offsets, const float *samples, int64_t n_samples,
                  const sdmm_mixtures *mix, const sdmm_fit_opts *opts, double *F_out,
                  double *g_alpha, double *g_mu_pos, double *g_delta, double *g_L,
                  int32_t *cell_status, void *workspace, size_t workspace_bytes, void *stream);

/*
 * sdmm_mixture_from_params -- the unconstrained parameterisation for gradient-based
 * refinement (the adjoint is derived from the MAP objective of Sec. 4.3; the paper itself
 * has no gradients): per cell pi = softmax(alpha); mu_dir = exp_{mu0}(delta) with the
 * exp map of Sec. 3.1 in the frame of mu0 (the fit's frame); mu_pos copied;
 * Sigma = L L^T.
 * alpha [device] float64[n_cells*K]; mu_dir0 [device] float64[n_cells*K*3] (normalised
 * here); delta [device] float64[n_cells*K*2]; mu_pos [device] float64[n_cells*K*3];
 * L [device] float64[n_cells*K*15] packed lower-triangular, row-major (index d(d+1)/2+e).
 * out: mixtures of the same n_cells and K, written (caller-owned device arrays).
 * jac_out [device] float64[n_cells*K*4] or NULL: the 2x2 Jacobian (row-major) of
 * delta -> log_{mu_dir}(exp_{mu0}(delta)) (the first-order transfer of Sec. 3.4 at
 * nu = delta), for sdmm_grad_to_params. Returns SDMM_EINVAL on bad sizes or NULL arrays.
 */
int sdmm_mixture_from_params(int32_t n_cells, int32_t K, const double *alpha, const double *mu_dir0,
                             const double *delta, const double *mu_pos, const double *L,
                             const sdmm_mixtures *out, double *jac_out, void *stream);

/*
 * sdmm_params_from_mixture -- the refinement parameters of a mixture: alpha = log pi and
 * L = the packed Cholesky factor of Sigma (positive pivots); delta = 0 and mu_dir0 =
 * mean_dir, mu_pos = mean_pos are the caller's to set. alpha [device] float64[n_cells*K],
 * L [device] float64[n_cells*K*15], cell_status [device] int32[n_cells] or NULL
 * (0, or SDMM_CELL_BAD_PARAMS for a cell with a non-SPD Sigma or a weight <= 0; its
 * L rows are 0 and alpha may be -inf).
 */
int sdmm_params_from_mixture(const sdmm_mixtures *mix, double *alpha, double *L, int32_t *cell_status,
                             void *stream);

/*
 * sdmm_grad_to_params -- pulls the gradients of sdmm_fit_grad (taken at the mixture that
 * sdmm_mixture_from_params produced) back onto (delta, L), in place:
 * g_delta := J^T g_delta; the columns e of g_L with L_ee < 0 change sign (sdmm_fit_grad
 * differentiates with respect to the Cholesky factor of Sigma, whose pivots are positive).
 * The alpha and mu_pos gradients need no change. Arrays as in sdmm_mixture_from_params;
 * g_delta [device] float64[n_cells*K*2], g_L [device] float64[n_cells*K*15].
 */
int sdmm_grad_to_params(int32_t n_cells, int32_t K, const double *L, const double *jac, double *g_delta,
                        double *g_L, void *stream);

/* ---- measurement ---- */

#define SDMM_TIMER_ESTEP 0   /* the E-step statistics pass of sdmm_fit_mixtures */
#define SDMM_TIMER_MSTEP 1   /* the M-step pass of sdmm_fit_mixtures */
#define SDMM_TIMER_QUERY 2   /* sdmm_condition_sample_pdf */
#define SDMM_TIMER_GRAD 3    /* the adjoint pass of sdmm_fit_grad */
#define SDMM_TIMER_ACCURATE 4 /* the second E-step pass of SDMM_FLAG_ACCURATE_SIGMA */
#define SDMM_TIMER_PRODUCT 5  /* sdmm_product_sample */
#define SDMM_TIMER_TREE 6     /* the first point-location launch of sdmm_tree_refine (every
                                 sample walked from the root) */
#define SDMM_TIMER_STEPWISE 7 /* the stepwise-EM kernel of SDMM_SCHED_STEPWISE */

/* Enables (1) or disables (0) HIP-event timing: while enabled, every eager launch of
 * the kernel classes above is bracketed by a pair of events recorded on its stream
 * (launches inside a hipGraph capture are not). Process-wide; returns SDMM_OK. */
int sdmm_timing_enable(int enable);

/* Waits for the recorded events of one class and returns the summed kernel time in
 * milliseconds and the number of launches; reset != 0 frees the records. Host call;
 * synchronises on the recorded events. SDMM_EINVAL for an unknown class. */
int sdmm_timing_read(int kernel_class, double *total_ms, int64_t *launches, int reset);

/* Device microbenchmark of the vector FMA rate the library's code generation reaches
 * (measurement support, not a step of the method): n_groups work groups of 256 threads,
 * each thread running `iters` rounds of 16 independent FMA chains in FP32 (bits = 32,
 * built without packed FP32 like every kernel here) or FP64 (bits = 64), and storing its
 * sum in out (device memory, n_groups * 256 floats or doubles). The work is
 * n_groups * 256 * iters * 16 FMAs (2 flop each). Writes the kernel time in milliseconds
 * (HIP events on the stream; the call synchronises on them) to *ms. SDMM_EINVAL for other
 * bits, n_groups < 1, iters < 1 or a null pointer. */
int sdmm_probe_fma(int32_t bits, int32_t n_groups, int32_t iters, void *out, double *ms, void *stream);

/* ---- helpers ---- */

/* Static description of an SDMM_OK / SDMM_E* code. */
const char *sdmm_status_string(int code);

/* Library version string. */
const char *sdmm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SDMM_H */
