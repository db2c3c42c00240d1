"""Pins for the oracle's EM: statistics (Sec. 3.2), the M-step with the first-order
covariance transfer (Sec. 3.4), Robbins-Monro averaging and MAP updates (Sec. 4.3).

Checks are against an independent textbook weighted MAP-EM (Euclidean special case),
closed forms (K = 1), invariances the method must have, and the MAP objective."""
import json
import os

import numpy as np
import pytest
from scipy.stats import multivariate_normal

from paper_2111_13094_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _tri(d, e):
    return d * (d + 1) // 2 + e


def _unpack(c):
    S = np.zeros((5, 5))
    for d in range(5):
        for e in range(d + 1):
            S[d, e] = S[e, d] = c[_tri(d, e)]
    return S


def _pack(S):
    return np.array([S[d, e] for d in range(5) for e in range(d + 1)])


def _single_cell(n=2048, K=16, seed=3, parallax=True, zero_frac=0.1, sigma=1.5):
    wl = synth.workload("single", seed=seed)
    b = synth.make_batch(seed + 7, [n], wl["box_lo"], wl["box_size"], wl["lobes"], parallax=parallax,
                         weight_sigma=sigma, zero_frac=zero_frac)
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], K)
    return b, mix


# --- golden constants -------------------------------------------------------

def test_paper_constants(orc):
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    o = orc.Opts(K=g["K"]).to_c()
    assert o.prior_q == pytest.approx(g["prior_q"], rel=1e-15)
    assert o.prior_a == pytest.approx(g["prior_a"], rel=1e-15)
    assert list(o.prior_b) == pytest.approx(g["prior_b_diag"], rel=1e-14)
    opts = orc.Opts(K=16, eta_mode=1, rm_alpha=g["rm_alpha"], rm_beta=g["rm_beta"])
    for j, e in enumerate(g["eta_j_0_to_5"]):
        assert orc.eta(opts, j) == pytest.approx(e, rel=1e-15)
    # the Robbins-Monro conditions of Sec. 4.3: sum eta = inf, sum eta^2 < inf needs alpha in (0.5, 1];
    # alpha = 0.5 sits at the boundary (sum eta^2 diverges logarithmically), as the paper chooses.
    from scipy.stats import chi2
    assert chi2.ppf(0.9, 3) == pytest.approx(g["chi2_3_inv_0p9"], rel=1e-7)
    assert synth.CHI2_3_INV_090 == pytest.approx(g["chi2_3_inv_0p9"], rel=1e-7)
    mix = synth.initial_mixtures(np.zeros((1, 3)), np.ones((1, 3)), 16)
    assert mix["cov"][0] == pytest.approx(g["init_sigma2_dir"], rel=1e-15)


# --- P3 responsibilities ------------------------------------------------------

def test_responsibilities_sum_to_one(orc):
    b, mix = _single_cell(256)
    o = orc.Opts(K=16)
    for i in range(0, 256, 7):
        r = orc.responsibilities(o, b.samples[0:3, i], b.samples[3:6, i], mix)
        assert abs(r.sum() - 1.0) < 1e-14 and (r >= 0).all()


# --- P4 Euclidean special case = textbook weighted MAP-EM ---------------------

def _textbook_step(X, w, pi, mu, Sig, beta, q, a, B):
    """Weighted MAP-EM step of a Gaussian mixture in R^5 with a Dirichlet prior on the
    weights and an inverse-Wishart-type prior on the covariances (Gauvain and Lee)."""
    K = pi.size
    logp = np.stack([np.log(pi[k]) + multivariate_normal(mu[k], Sig[k]).logpdf(X) for k in range(K)], 1)
    r = np.exp(logp - logp.max(1, keepdims=True))
    r /= r.sum(1, keepdims=True)
    W = w.sum()
    wr = w[:, None] * r
    N0 = wr.sum(0) / W
    mu_new = (wr.T @ X) / wr.sum(0)[:, None]
    Sig_new = np.zeros_like(Sig)
    for k in range(K):
        D = X - mu_new[k]
        Sig_new[k] = ((wr[:, k, None] * D).T @ D / W + beta * np.diag(B)) / (N0[k] + beta * a)
    pi_new = (N0 + beta * q) / (N0.sum() + K * beta * q)
    return pi_new, mu_new, Sig_new


def _euclid_problem(seed=11, n=1500, K=4):
    rng = np.random.default_rng(seed)
    centres = rng.normal(size=(K, 5)) * 2.0
    lab = rng.integers(0, K, n)
    X = centres[lab] + rng.normal(size=(n, 5)) * 0.5
    w = np.exp(rng.normal(size=n))
    w[rng.random(n) < 0.1] = 0.0
    smp = np.zeros((7, n), dtype=np.float32)
    smp[0:2] = X[:, 0:2].T
    smp[3:6] = X[:, 2:5].T
    smp[6] = w
    X = np.concatenate([smp[0:2].T, smp[3:6].T], 1).astype(np.float64)
    w = smp[6].astype(np.float64)
    pi = np.full(K, 1.0 / K)
    mu = X[rng.choice(n, K, replace=False)]
    Sig = np.stack([np.eye(5)] * K)
    mix = {"pi": pi.copy(), "mu_dir": np.concatenate([mu[:, 0:2], np.zeros((K, 1))], 1).ravel(),
           "mu_pos": mu[:, 2:5].copy().ravel(), "cov": np.concatenate([_pack(S) for S in Sig])}
    return smp, X, w, (pi, mu, Sig), mix


def test_euclidean_mode_equals_textbook_map_em(orc):
    smp, X, w, (pi, mu, Sig), mix = _euclid_problem()
    K = pi.size
    beta = 0.3
    opts = orc.Opts(K=K, iters=1, euclidean=1, prior_mode=1, prior_scale=beta, min_samples=16)
    o = opts.to_c()
    B = np.array(o.prior_b)
    st = orc.new_state(1, K)
    off = np.array([0, X.shape[0]])
    for it in range(6):
        pi, mu, Sig = _textbook_step(X, w, pi, mu, Sig, beta, o.prior_q, o.prior_a, B)
        status = orc.fit(opts, off, smp, mix, st)
        assert status[0] == 0
        got_mu = np.concatenate([mix["mu_dir"].reshape(K, 3)[:, :2], mix["mu_pos"].reshape(K, 3)], 1)
        assert np.allclose(mix["pi"], pi, rtol=1e-10, atol=1e-14)
        assert np.allclose(got_mu, mu, rtol=1e-10, atol=1e-12)
        got_S = np.stack([_unpack(c) for c in mix["cov"].reshape(K, 15)])
        assert np.allclose(got_S, Sig, rtol=1e-9, atol=1e-13)


def test_euclidean_mode_objective_is_monotone_and_stationary(orc):
    smp, X, w, _, mix = _euclid_problem(seed=12, n=1200, K=3)
    K = 3
    beta = 0.05
    opts = orc.Opts(K=K, iters=1, euclidean=1, prior_mode=1, prior_scale=beta)
    st = orc.new_state(1, K)
    off = np.array([0, X.shape[0]])
    F = [orc.objective(opts, smp, 0, X.shape[0], mix, beta)]
    for it in range(400):
        orc.fit(opts, off, smp, mix, st)
        F.append(orc.objective(opts, smp, 0, X.shape[0], mix, beta))
    F = np.array(F)
    assert (np.diff(F) >= -1e-12 * np.abs(F[1:])).all(), np.diff(F).min()
    g = orc.grad(opts, smp, 0, X.shape[0], mix, beta)
    for key in ("alpha", "mu_pos", "delta", "L"):
        assert np.abs(g[key]).max() < 1e-8, (key, np.abs(g[key]).max())


# --- P5 K = 1 closed forms ----------------------------------------------------

def test_single_component_closed_forms(orc):
    rng = np.random.default_rng(21)
    n = 3000
    lobe = _unit(np.array([0.2, -0.7, 0.5]))
    smp = np.zeros((7, n), dtype=np.float32)
    smp[0:3] = synth.sample_vmf(rng, np.tile(lobe, (n, 1)), np.full(n, 4.0)).T
    smp[3:6] = rng.random((3, n))
    smp[6] = synth.draw_weights(rng, n)
    mix = synth.initial_mixtures(np.zeros((1, 3)), np.ones((1, 3)), 1)
    beta = 0.01
    opts = orc.Opts(K=1, iters=1, prior_mode=1, prior_scale=beta)
    o = opts.to_c()
    st = orc.new_state(1, 1)
    orc.fit(opts, np.array([0, n]), smp, mix, st)
    w = smp[6].astype(np.float64)
    P = smp[3:6].T.astype(np.float64)
    W = w.sum()
    mean = (w[:, None] * P).sum(0) / W
    assert mix["pi"][0] == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(mix["mu_pos"], mean, rtol=1e-12)
    D = P - mean
    scatter = (w[:, None] * D).T @ D / W
    Sxx = (scatter + beta * np.diag(o.prior_b[2:5])) / (1.0 + beta * o.prior_a)
    S = _unpack(mix["cov"])
    assert np.allclose(S[2:, 2:], Sxx, rtol=1e-11)
    # directional fixed point = weighted Karcher mean: sum_i w_i log_mu(w_i) = 0, written in
    # world coordinates as theta_i (w_i - cos theta_i mu) / sin theta_i.
    for it in range(100):
        orc.fit(opts, np.array([0, n]), smp, mix, st)
    mu = mix["mu_dir"]
    Wd = smp[0:3].T.astype(np.float64)
    cos = Wd @ mu
    proj = Wd - cos[:, None] * mu
    sin = np.linalg.norm(proj, axis=1)
    th = np.arctan2(sin, cos)
    v = (w * th / sin)[:, None] * proj
    assert np.linalg.norm(v.sum(0)) / W < 1e-10


# --- P10 invariances ----------------------------------------------------------

def _fit_copy(orc, opts, off, smp, mix, st=None):
    mix = synth.copy_mix(mix)
    st = orc.new_state(off.size - 1, opts.K) if st is None else {k: v.copy() for k, v in st.items()}
    s = orc.fit(opts, off, smp, mix, st)
    return mix, st, s


def test_weight_scale_invariance(orc):
    b, mix = _single_cell(1024)
    opts = orc.Opts(K=16, iters=3)
    off = b.offsets
    m1, s1, _ = _fit_copy(orc, opts, off, b.samples, mix)
    smp = b.samples.copy()
    smp[6] *= 4.0  # exact in float32
    m2, s2, _ = _fit_copy(orc, opts, off, smp, mix)
    for k in m1:
        assert np.allclose(m1[k], m2[k], rtol=1e-13, atol=1e-15)


def test_zero_weight_samples_are_inert(orc):
    b, mix = _single_cell(1024, zero_frac=0.3)
    opts = orc.Opts(K=16, iters=3)
    m1, s1, _ = _fit_copy(orc, opts, b.offsets, b.samples, mix)
    keep = b.samples[6] > 0
    smp = np.ascontiguousarray(b.samples[:, keep])
    m2, s2, _ = _fit_copy(orc, opts, np.array([0, smp.shape[1]]), smp, mix)
    for k in m1:
        assert np.array_equal(m1[k], m2[k]), k


def test_sample_permutation_invariance(orc):
    b, mix = _single_cell(1024)
    opts = orc.Opts(K=16, iters=3)
    m1, _, _ = _fit_copy(orc, opts, b.offsets, b.samples, mix)
    perm = np.random.default_rng(5).permutation(b.samples.shape[1])
    m2, _, _ = _fit_copy(orc, opts, b.offsets, np.ascontiguousarray(b.samples[:, perm]), mix)
    for k in m1:
        assert np.allclose(m1[k], m2[k], rtol=1e-10, atol=1e-12), k


def _world_tangent_cov(mu, cov_packed, orc):
    """Directional covariance and direction-position cross covariance as world-space
    tangent vectors (independent of the frame chosen about mu)."""
    R = orc.frame(mu)
    E = R[:2].T  # 3x2, columns t1, t2
    S = _unpack(cov_packed)
    return E @ S[:2, :2] @ E.T, E @ S[:2, 2:]


def test_global_rotation_equivariance(orc):
    """Rotating every direction and every directional mean rotates the fitted model
    (world-space means and tangent covariances) and leaves pdf values unchanged."""
    b, mix = _single_cell(1500)
    opts = orc.Opts(K=16, iters=4)
    ang = 0.7
    Q = np.array([[np.cos(ang), -np.sin(ang), 0], [np.sin(ang), np.cos(ang), 0], [0, 0, 1]])
    Q = Q @ np.array([[1, 0, 0], [0, np.cos(0.4), -np.sin(0.4)], [0, np.sin(0.4), np.cos(0.4)]])
    m1, _, _ = _fit_copy(orc, opts, b.offsets, b.samples, mix)
    smp = b.samples.copy()
    smp[0:3] = (Q @ b.samples[0:3].astype(np.float64)).astype(np.float32)
    # rotating float32 directions introduces float32 rounding: compare the unrotated fit
    # on the same rounded directions rotated back.
    back = np.ascontiguousarray(b.samples.copy())
    back[0:3] = (Q.T @ smp[0:3].astype(np.float64)).astype(np.float32)
    m1, _, _ = _fit_copy(orc, opts, b.offsets, back, mix)
    mixr = synth.copy_mix(mix)
    mixr["mu_dir"] = (mix["mu_dir"].reshape(-1, 3) @ Q.T).ravel()
    m2, _, _ = _fit_copy(orc, opts, b.offsets, smp, mixr)
    assert np.allclose(m1["pi"], m2["pi"], rtol=1e-5)
    assert np.allclose(m1["mu_dir"].reshape(-1, 3) @ Q.T, m2["mu_dir"].reshape(-1, 3), atol=1e-5)
    assert np.allclose(m1["mu_pos"], m2["mu_pos"], atol=1e-5)
    for k in range(16):
        A1, X1 = _world_tangent_cov(m1["mu_dir"][3 * k:3 * k + 3], m1["cov"][15 * k:15 * k + 15], orc)
        A2, X2 = _world_tangent_cov(m2["mu_dir"][3 * k:3 * k + 3], m2["cov"][15 * k:15 * k + 15], orc)
        assert np.allclose(Q @ A1 @ Q.T, A2, atol=1e-5 * np.abs(A1).max())
        assert np.allclose(Q @ X1, X2, atol=1e-5 * max(np.abs(X1).max(), 1e-6))
    x = np.array([0.4, 0.5, 0.6])
    dirs = _unit(np.random.default_rng(3).normal(size=(50, 3)))
    p1 = orc.pdf(16, m1, x[None], np.array([0]), dirs[None])
    p2 = orc.pdf(16, m2, x[None], np.array([0]), (dirs @ Q.T)[None])
    assert np.allclose(p1, p2, rtol=1e-4)


def test_exact_rotation_equivariance_of_pdf(orc):
    """Evaluating a fixed model: rotating the directional means and the query directions
    by a rotation about z that maps the frame onto itself leaves pdf values unchanged to
    rounding (1e-10)."""
    b, mix = _single_cell(1000)
    opts = orc.Opts(K=16, iters=3)
    m1, _, _ = _fit_copy(orc, opts, b.offsets, b.samples, mix)
    x = np.array([0.3, 0.6, 0.4])
    dirs = _unit(np.random.default_rng(4).normal(size=(64, 3)))
    p1 = orc.pdf(16, m1, x[None], np.array([0]), dirs[None])
    # a quarter turn about z permutes coordinates exactly
    Q = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    m2 = synth.copy_mix(m1)
    m2["mu_dir"] = (m1["mu_dir"].reshape(-1, 3) @ Q.T).ravel()
    # Sigma is stored in each mean's frame; re-express it in the rotated mean's frame
    for k in range(16):
        R1 = orc.frame(m1["mu_dir"][3 * k:3 * k + 3])
        R2 = orc.frame(m2["mu_dir"][3 * k:3 * k + 3])
        G = R2[:2] @ Q @ R1[:2].T  # 2x2 frame change
        T = np.eye(5)
        T[:2, :2] = G
        S = _unpack(m1["cov"][15 * k:15 * k + 15])
        m2["cov"][15 * k:15 * k + 15] = _pack(T @ S @ T.T)
    p2 = orc.pdf(16, m2, x[None], np.array([0]), (dirs @ Q.T)[None])
    assert np.allclose(p1, p2, rtol=1e-10, atol=1e-14)


def test_cell_independence(orc):
    wl = synth.workload("cells4k", scale=8 / 4096)
    b = synth.workload_batch(wl)
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    C = wl["grid"].n_cells
    opts = orc.Opts(K=16, iters=2)
    mall, sall, stat = _fit_copy(orc, opts, b.offsets, b.samples, mix)
    for c in range(C):
        i0, i1 = b.offsets[c], b.offsets[c + 1]
        sub = np.ascontiguousarray(b.samples[:, i0:i1])
        mc = {k: np.ascontiguousarray(v.reshape(C, -1)[c]) for k, v in mix.items()}
        mm, ss, s = _fit_copy(orc, opts, np.array([0, i1 - i0]), sub, mc)
        assert s[0] == stat[c]
        for k in mm:
            assert np.array_equal(mm[k], mall[k].reshape(C, -1)[c])


# --- gating and status --------------------------------------------------------

def test_gating_statuses_leave_cells_untouched(orc):
    wl = synth.workload("cells4k", scale=8 / 4096)
    b = synth.workload_batch(wl)
    C = wl["grid"].n_cells
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    smp = b.samples.copy()
    off = b.offsets
    smp[6, off[1] + 3] = np.nan                 # cell 1: bad input
    smp[6, off[2] + 5] = -1.0                   # cell 2: negative weight
    smp[6, off[3]:off[4]] = 0.0                 # cell 3: all weights zero -> too few
    smp[6, off[4] + 20:off[5]] = 0.0            # cell 4: 20 positive samples at most
    smp[6, off[4]:off[4] + 20] = 1.0
    cov_bad = mix["cov"].reshape(C, 16, 15).copy()
    cov_bad[5, 3, 0] = -1.0                     # cell 5: non-SPD covariance
    mix["cov"] = cov_bad.ravel()
    opts = orc.Opts(K=16, iters=2)
    m, s, stat = _fit_copy(orc, opts, off, smp, mix)
    assert stat[1] == orc.BAD_INPUT and stat[2] == orc.BAD_INPUT
    assert stat[3] == orc.SKIPPED_FEW
    assert stat[4] & (orc.SKIPPED_FEW | orc.SKIPPED_ZERO_W) == 0
    assert stat[5] == orc.BAD_PARAMS
    for c in (1, 2, 3, 5):
        for k in m:
            assert np.array_equal(m[k].reshape(C, -1)[c], mix[k].reshape(C, -1)[c])
        assert s["step"][c] == 0
    assert stat[0] in (0, orc.DEAD_COMPONENT)
    m0, _, _ = _fit_copy(orc, opts, off, b.samples, synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16))
    for k in m:  # cell 0 (clean) identical to a clean run
        assert np.array_equal(m[k].reshape(C, -1)[0], m0[k].reshape(C, -1)[0])
    smp2 = smp.copy()
    smp2[6, off[4]:off[4] + 20] = 0.0
    smp2[6, off[4]:off[4] + 15] = 1.0
    _, _, stat2 = _fit_copy(orc, opts, off, smp2, synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16))
    assert stat2[4] == orc.SKIPPED_FEW


# --- P11 Robbins-Monro special cases -----------------------------------------

def test_eta_one_equals_independent_single_batch_step(orc):
    wl = synth.workload("single", scale=1024 / 16384)
    b0 = synth.workload_batch(wl, 0)
    b1 = synth.workload_batch(wl, 1)
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    opts = orc.Opts(K=16, iters=1, eta_mode=0, eta=1.0)
    m, st, _ = _fit_copy(orc, opts, b0.offsets, b0.samples, mix)
    m_a, _, _ = _fit_copy(orc, opts, b1.offsets, b1.samples, m, st)
    m_b, _, _ = _fit_copy(orc, opts, b1.offsets, b1.samples, m)  # fresh state (j = 0)
    for k in m_a:
        assert np.array_equal(m_a[k], m_b[k]), k


def test_repeated_batch_with_small_eta_reaches_the_batch_em_fixed_point(orc):
    b, mix = _single_cell(1024, K=4, parallax=False)
    mix = synth.initial_mixtures(np.zeros((1, 3)), np.ones((1, 3)), 4)
    beta = 1e-3
    batch = orc.Opts(K=4, iters=600, eta_mode=0, eta=1.0, prior_mode=1, prior_scale=beta)
    mb, _, _ = _fit_copy(orc, batch, b.offsets, b.samples, mix)
    step = orc.Opts(K=4, iters=1500, eta_mode=0, eta=0.1, prior_mode=1, prior_scale=beta)
    ms, _, _ = _fit_copy(orc, step, b.offsets, b.samples, mix)
    assert np.allclose(mb["pi"], ms["pi"], atol=1e-7)
    assert np.allclose(mb["mu_dir"], ms["mu_dir"], atol=1e-7)
    assert np.allclose(mb["mu_pos"], ms["mu_pos"], atol=1e-7)
    assert np.allclose(mb["cov"], ms["cov"], atol=1e-7)


# --- P13 tangent-mode monotonicity (first-order M-step is not exact) ---------

def test_tangent_mode_objective_nearly_monotone(orc):
    b, mix = _single_cell(2048, parallax=True)
    beta = 1.0 / 2048
    opts = orc.Opts(K=16, iters=1, prior_mode=1, prior_scale=beta)
    st = orc.new_state(1, 16)
    n = b.samples.shape[1]
    F = [orc.objective(opts, b.samples, 0, n, mix, beta)]
    for it in range(30):
        orc.fit(opts, b.offsets, b.samples, mix, st)
        F.append(orc.objective(opts, b.samples, 0, n, mix, beta))
    F = np.array(F)
    dips = np.diff(F) / np.abs(F[1:])
    assert dips.min() >= -1e-6, dips.min()
    assert F[-1] > F[0]


def test_malformed_offsets_reject_the_whole_batch(orc):
    """Offsets that decrease anywhere, start below 0 or end beyond the sample count make
    every cell report BAD_INPUT and leave every parameter unchanged."""
    wl = synth.workload("cells4k", scale=8 / 4096)
    b = synth.workload_batch(wl)
    C = wl["grid"].n_cells
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    N = b.samples.shape[1]
    bad = []
    o1 = b.offsets.copy()
    o1[3], o1[4] = o1[4], o1[3]
    bad.append(o1)
    o2 = b.offsets.copy()
    o2[-1] = N + 1
    bad.append(o2)
    o3 = b.offsets.copy()
    o3[0] = -1
    bad.append(o3)
    for off in bad:
        m, s, stat = _fit_copy(orc, orc.Opts(K=16), off, b.samples, mix)
        assert (stat == orc.BAD_INPUT).all()
        for k in m:
            assert np.array_equal(m[k], mix[k])
        assert (s["step"] == 0).all()
    # a prefix of the array is fine: samples after the last offset are not used
    o4 = b.offsets.copy()
    o4[-1] = o4[-2]
    m, s, stat = _fit_copy(orc, orc.Opts(K=16), o4, b.samples, mix)
    assert stat[-1] == orc.SKIPPED_FEW and (stat[:-1] & orc.BAD_INPUT == 0).all()


# --- P12 accurate covariance update (Sec. 3.2, second pass in the new tangent space) ---

def _geodesic_coords(Wd, P, mu, mx, basis_seed):
    """Tangent coordinates of unit directions about `mu` from their geodesic distance and
    direction, in an orthonormal tangent basis chosen independently of the oracle's frame."""
    cos = Wd @ mu
    proj = Wd - cos[:, None] * mu
    sin = np.linalg.norm(proj, axis=1)
    th = np.arctan2(sin, cos)
    e1 = _unit(np.cross(mu, np.random.default_rng(basis_seed).normal(size=3)))
    e2 = np.cross(mu, e1)
    nu = (th / sin)[:, None] * np.stack([proj @ e1, proj @ e2], 1)
    return np.concatenate([nu, P - mx], 1)


def _accurate_problem(n=3000, kappa=4.0, offset=0.7, K=1, seed=21):
    rng = np.random.default_rng(seed)
    lobes = [_unit(np.array([0.2, -0.7, 0.5])), _unit(np.array([-0.6, 0.1, 0.4])), _unit(np.array([0.3, 0.8, 0.2]))]
    lab = rng.integers(0, K, n)
    smp = np.zeros((7, n), dtype=np.float32)
    smp[0:3] = synth.sample_vmf(rng, np.stack([lobes[k] for k in lab]), np.full(n, kappa)).T
    smp[3:6] = rng.random((3, n))
    smp[3] += 0.8 * smp[0]  # direction-position coupling, so the cross block is not zero
    smp[6] = synth.draw_weights(rng, n)
    mix = synth.initial_mixtures(np.zeros((1, 3)), np.ones((1, 3)), K)
    mud = mix["mu_dir"].reshape(K, 3)
    for k in range(K):
        ax = _unit(np.cross(lobes[k], [1.0, 0.0, 0.0]))
        mud[k] = np.cos(offset) * lobes[k] + np.sin(offset) * ax
    return smp, mix


def test_accurate_sigma_single_component_is_the_scatter_about_the_new_mean(orc):
    """K = 1: every responsibility is 1, so the accurate update is the weighted second
    moment of the samples' geodesic tangent coordinates about the new mean, plus the
    prior. Compared up to a rotation of the tangent basis (eigenvalues of the 5x5 matrix)
    and exactly in the positional block. The first-order transfer is visibly off here
    (the initial mean is 0.7 rad from the lobe)."""
    smp, mix0 = _accurate_problem()
    n = smp.shape[1]
    beta = 0.01
    gaps = {}
    for acc in (1, 0):
        mix = synth.copy_mix(mix0)
        opts = orc.Opts(K=1, iters=1, prior_mode=1, prior_scale=beta, accurate_sigma=acc)
        o = opts.to_c()
        st = orc.new_state(1, 1)
        assert orc.fit(opts, np.array([0, n]), smp, mix, st)[0] == 0
        w = smp[6].astype(np.float64)
        Y = _geodesic_coords(smp[0:3].T.astype(np.float64), smp[3:6].T.astype(np.float64), mix["mu_dir"],
                             mix["mu_pos"], 5)
        scatter = (w[:, None] * Y).T @ Y / w.sum()
        S = _unpack(mix["cov"]) * (1.0 + beta * o.prior_a) - beta * np.diag(o.prior_b)
        ev, ev_ref = np.linalg.eigvalsh(S), np.linalg.eigvalsh(scatter)
        gaps[acc] = np.abs(ev - ev_ref).max() / ev_ref.max()
        assert np.allclose(S[2:, 2:], scatter[2:, 2:], rtol=1e-12, atol=1e-15)
    assert gaps[1] < 1e-12, gaps
    assert gaps[0] > 1e-3, gaps


def test_accurate_sigma_responsibilities_come_from_the_new_means(orc):
    """K = 3 on the sphere: each component's accurate covariance is the second moment of
    the geodesic coordinates about its new mean, weighted by w r' with r' the
    responsibilities under the new weights and means and the previous covariances, and
    normalised by the same weights."""
    K = 3
    smp, mix0 = _accurate_problem(n=2400, kappa=10.0, offset=0.3, K=K, seed=8)
    n = smp.shape[1]
    beta = 0.02
    opts = orc.Opts(K=K, iters=1, prior_mode=1, prior_scale=beta, accurate_sigma=1)
    o = opts.to_c()
    mix = synth.copy_mix(mix0)
    st = orc.new_state(1, K)
    assert orc.fit(opts, np.array([0, n]), smp, mix, st)[0] == 0
    mid = dict(mix, cov=mix0["cov"].copy())  # new weights and means, previous covariances
    r = np.stack([orc.responsibilities(opts, smp[0:3, i].astype(np.float64), smp[3:6, i].astype(np.float64), mid)
                  for i in range(n)])
    w = smp[6].astype(np.float64)
    W = w.sum()
    for k in range(K):
        mu, mx = mix["mu_dir"].reshape(K, 3)[k], mix["mu_pos"].reshape(K, 3)[k]
        Y = _geodesic_coords(smp[0:3].T.astype(np.float64), smp[3:6].T.astype(np.float64), mu, mx, k)
        wr = w * r[:, k]
        scatter = (wr[:, None] * Y).T @ Y / W
        S = _unpack(mix["cov"].reshape(K, 15)[k]) * (beta * o.prior_a + wr.sum() / W) - beta * np.diag(o.prior_b)
        ev, ev_ref = np.linalg.eigvalsh(S), np.linalg.eigvalsh(scatter)
        assert np.abs(ev - ev_ref).max() < 1e-11 * ev_ref.max(), (k, ev, ev_ref)
        assert np.allclose(S[2:, 2:], scatter[2:, 2:], rtol=1e-11, atol=1e-15)
        assert st["s0"][k] == pytest.approx(wr.sum(), rel=1e-12)


def _textbook_ecm_step(X, w, pi, mu, Sig, beta, q, a, B):
    """One cycle of multi-cycle ECM for a weighted MAP Gaussian mixture in R^5 (Meng and
    Rubin 1993): E-step, weights and means, a second E-step under the new weights and
    means, then the covariances about the new means with those responsibilities."""
    K = pi.size

    def resp(pi, mu, Sig):
        logp = np.stack([np.log(pi[k]) + multivariate_normal(mu[k], Sig[k]).logpdf(X) for k in range(K)], 1)
        r = np.exp(logp - logp.max(1, keepdims=True))
        return r / r.sum(1, keepdims=True)

    W = w.sum()
    wr = w[:, None] * resp(pi, mu, Sig)
    N0 = wr.sum(0) / W
    mu_new = (wr.T @ X) / wr.sum(0)[:, None]
    pi_new = (N0 + beta * q) / (N0.sum() + K * beta * q)
    wr2 = w[:, None] * resp(pi_new, mu_new, Sig)
    Sig_new = np.zeros_like(Sig)
    for k in range(K):
        D = X - mu_new[k]
        Sig_new[k] = ((wr2[:, k, None] * D).T @ D / W + beta * np.diag(B)) / (wr2[:, k].sum() / W + beta * a)
    return pi_new, mu_new, Sig_new


def test_accurate_sigma_is_the_textbook_ecm_cycle_in_euclidean_mode(orc):
    """Euclidean coordinates: moving the frame is a translation, so the accurate update is
    one cycle of multi-cycle ECM, written here independently."""
    smp, X, w, (pi, mu, Sig), mix = _euclid_problem(seed=13)
    K = pi.size
    beta = 0.3
    opts = orc.Opts(K=K, iters=1, euclidean=1, prior_mode=1, prior_scale=beta, accurate_sigma=1)
    o = opts.to_c()
    st = orc.new_state(1, K)
    for it in range(4):
        pi, mu, Sig = _textbook_ecm_step(X, w, pi, mu, Sig, beta, o.prior_q, o.prior_a, np.array(o.prior_b))
        assert orc.fit(opts, np.array([0, X.shape[0]]), smp, mix, st)[0] == 0
        got_mu = np.concatenate([mix["mu_dir"].reshape(K, 3)[:, :2], mix["mu_pos"].reshape(K, 3)], 1)
        got_S = np.stack([_unpack(c) for c in mix["cov"].reshape(K, 15)])
        assert np.allclose(mix["pi"], pi, rtol=1e-10, atol=1e-14)
        assert np.allclose(got_mu, mu, rtol=1e-10, atol=1e-12)
        assert np.allclose(got_S, Sig, rtol=1e-9, atol=1e-13)


def test_accurate_sigma_objective_is_monotone_in_euclidean_mode(orc):
    """Every ECM cycle maximises the penalised objective over a block of parameters with
    the others fixed, so the objective never decreases."""
    smp, X, w, _, mix = _euclid_problem(seed=12, n=1200, K=3)
    beta = 0.05
    opts = orc.Opts(K=3, iters=1, euclidean=1, prior_mode=1, prior_scale=beta, accurate_sigma=1)
    st = orc.new_state(1, 3)
    off = np.array([0, X.shape[0]])
    F = [orc.objective(opts, smp, 0, X.shape[0], mix, beta)]
    for it in range(200):
        orc.fit(opts, off, smp, mix, st)
        F.append(orc.objective(opts, smp, 0, X.shape[0], mix, beta))
    F = np.array(F)
    assert (np.diff(F) >= -1e-12 * np.abs(F[1:])).all(), np.diff(F).min()
    assert F[-1] > F[0]


def test_accurate_sigma_needs_batch_steps(orc):
    smp, mix = _accurate_problem(n=64)
    st = orc.new_state(1, 1)
    for kw in ({"eta": 0.5}, {"eta_mode": 1}):
        with pytest.raises(ValueError):
            orc.fit(orc.Opts(K=1, accurate_sigma=1, **kw), np.array([0, 64]), smp, synth.copy_mix(mix), st)


def test_covariance_updates_naive_first_order_accurate(orc):
    """The comparison the paper draws for one component whose mean moves: reusing the
    old-frame covariance unchanged (naive), carrying it by the first-order Jacobian, and
    the accurate second pass. Against the accurate update (which the K = 1 pin ties to
    the geodesic scatter), the first-order transfer is several times closer than the
    naive update at every mean shift, and both errors grow with the shift."""
    rng = np.random.default_rng(21)
    n = 20000
    lobe = _unit(np.array([0.2, -0.7, 0.5]))
    smp = np.zeros((7, n), dtype=np.float32)
    smp[0:3] = synth.sample_vmf(rng, np.tile(lobe, (n, 1)), np.full(n, 16.0)).T
    smp[3:6] = rng.random((3, n))
    smp[3] += 0.8 * smp[0]
    smp[6] = synth.draw_weights(rng, n)
    beta = 0.01
    o = orc.Opts(K=1, prior_mode=1, prior_scale=beta).to_c()
    errs = []
    for delta in (0.1, 0.4, 1.2):
        mix0 = synth.initial_mixtures(np.zeros((1, 3)), np.ones((1, 3)), 1)
        ax = _unit(np.cross(lobe, [1.0, 0.0, 0.0]))
        mix0["mu_dir"][:] = np.cos(delta) * lobe + np.sin(delta) * ax
        out = {}
        for acc in (1, 0):
            mix = synth.copy_mix(mix0)
            orc.fit(orc.Opts(K=1, prior_mode=1, prior_scale=beta, accurate_sigma=acc), np.array([0, n]), smp, mix,
                    orc.new_state(1, 1))
            out[acc] = _unpack(mix["cov"])
        st = orc.cell_stats(orc.Opts(K=1), smp, 0, n, mix0)
        S0, S1, S2, W = st["S0"][0], st["S1"][0], _unpack(st["S2"][0]), st["W"]
        naive = (beta * np.diag(o.prior_b) + (S2 - np.outer(S1, S1) / S0) / W) / (beta * o.prior_a + S0 / W)
        A = out[1]
        e_naive = np.linalg.norm(naive - A) / np.linalg.norm(A)
        e_first = np.linalg.norm(out[0] - A) / np.linalg.norm(A)
        print(f"shift {delta}: naive {e_naive:.2e}, first-order {e_first:.2e}")
        assert e_first < e_naive / 5, (delta, e_first, e_naive)
        errs.append((e_naive, e_first))
    assert errs[0][0] < errs[1][0] < errs[2][0] and errs[0][1] < errs[1][1] < errs[2][1]


# --- P13 stepwise (per-sample) EM --------------------------------------------------------

def test_stepwise_single_component_is_the_exponentially_weighted_estimate(orc):
    """K = 1 in Euclidean coordinates with a constant eta: after the warm-start batch step
    the per-sample recursion must equal the exponentially weighted mean and covariance
    written out directly: the batch samples weigh (1 - eta)^j w_i, and the sample taken
    at step i weighs eta (1 - eta)^(j - i) w_i; Sigma = (beta B + C / W^) / (beta a + 1)
    with beta = eta (a mini-batch of one) and W^ the same weights' total."""
    rng = np.random.default_rng(31)
    n, eta = 300, 0.05
    X = rng.normal(size=(n, 5)) * np.array([0.3, 0.2, 1.0, 0.5, 0.7]) + 1.0
    w = np.exp(rng.normal(size=n)).astype(np.float32).astype(np.float64)
    w[rng.random(n) < 0.1] = 0.0
    smp = np.zeros((7, n), dtype=np.float32)
    smp[0:2] = X[:, 0:2].T
    smp[3:6] = X[:, 2:5].T
    smp[6] = w
    X = np.concatenate([smp[0:2].T, smp[3:6].T], 1).astype(np.float64)
    mix = {"pi": np.ones(1), "mu_dir": np.array([0.0, 0.0, 0.0]), "mu_pos": np.zeros(3),
           "cov": _pack(np.eye(5))}
    opts = orc.Opts(K=1, eta=eta, euclidean=1, min_samples=1)
    o = opts.to_c()
    st = orc.new_state(1, 1)
    assert orc.fit_stepwise(opts, np.array([0, n]), smp, mix, st)[0] == 0  # warm start: a batch step
    assert st["step"][0] == 1
    assert orc.fit_stepwise(opts, np.array([0, n]), smp, mix, st)[0] == 0  # one per-sample pass
    pos = np.nonzero(w > 0)[0]
    j = pos.size
    assert st["step"][0] == 1 + j
    lam = np.concatenate([w * (1 - eta) ** j, w[pos] * eta * (1 - eta) ** (j - 1 - np.arange(j))])
    Y = np.concatenate([X, X[pos]])
    mean = (lam[:, None] * Y).sum(0) / lam.sum()
    D = Y - mean
    Cw = (lam[:, None] * D).T @ D / lam.sum()
    Sig = (eta * np.diag(o.prior_b) + Cw) / (eta * o.prior_a + 1.0)
    got_mu = np.concatenate([mix["mu_dir"][:2], mix["mu_pos"]])
    assert np.allclose(got_mu, mean, rtol=1e-11, atol=1e-12)
    assert np.allclose(_unpack(mix["cov"]), Sig, rtol=1e-9, atol=1e-14)
    assert st["sw"][0] == pytest.approx(lam.sum(), rel=1e-12)


def test_stepwise_fresh_cells_take_a_batch_step(orc):
    b, mix = _single_cell(1024)
    opts = orc.Opts(K=16, eta=0.1)
    m1, s1, st1 = _fit_copy(orc, opts, b.offsets, b.samples, mix)
    m2 = synth.copy_mix(mix)
    s2 = orc.new_state(1, 16)
    st2 = orc.fit_stepwise(opts, b.offsets, b.samples, m2, s2)
    assert np.array_equal(st1, st2)
    for k in m1:
        assert np.array_equal(m1[k], m2[k]), k


def test_stepwise_skips_zero_weight_samples(orc):
    b, mix = _single_cell(512, zero_frac=0.3)
    opts = orc.Opts(K=16, eta_mode=1)
    m1, s1 = synth.copy_mix(mix), orc.new_state(1, 16)
    orc.fit_stepwise(opts, b.offsets, b.samples, m1, s1)
    orc.fit_stepwise(opts, b.offsets, b.samples, m1, s1)
    keep = b.samples[6] > 0
    smp = np.ascontiguousarray(b.samples[:, keep])
    m2, s2 = synth.copy_mix(mix), orc.new_state(1, 16)
    orc.fit_stepwise(opts, np.array([0, smp.shape[1]]), smp, m2, s2)
    orc.fit_stepwise(opts, np.array([0, smp.shape[1]]), smp, m2, s2)
    for k in m1:
        assert np.array_equal(m1[k], m2[k]), k
    assert s1["step"][0] == s2["step"][0] == 1 + keep.sum()


def test_stepwise_rejects_the_accurate_update(orc):
    b, mix = _single_cell(64)
    with pytest.raises(ValueError):
        orc.fit_stepwise(orc.Opts(K=16, accurate_sigma=1), b.offsets, b.samples, mix, orc.new_state(1, 16))


# --- default prior strength and solid-angle responsibilities (pins of two oracle branches)

def _k1_cell(rng, n, zero_frac, lo, size):
    """One cell of n samples for K = 1: a vMF lobe, positions uniform in the box, weights
    lognormal(0, 1.5) with a fraction set exactly to zero."""
    lobe = _unit(np.array([0.3, -0.5, 0.8]))
    smp = np.zeros((7, n), dtype=np.float32)
    smp[0:3] = synth.sample_vmf(rng, np.tile(lobe, (n, 1)), np.full(n, 6.0)).T
    smp[3:6] = (lo[:, None] + size[:, None] * rng.random((3, n))).astype(np.float32)
    w = np.exp(1.5 * rng.normal(size=n))
    w[rng.random(n) < zero_frac] = 0.0
    smp[6] = w.astype(np.float32)
    return smp


def test_default_prior_strength_is_eta_over_positive_count(orc):
    """Sec. 4.3 (MAP update with the prior strength of reading A12): with the default
    prior mode, beta_j = eta_j / M_j where M_j counts the batch's samples of positive
    weight. K = 1 makes every responsibility 1, so the positional block of the covariance
    has a closed form over two batches: after the first (eta = 1)
        Sigma_xx = (beta_0 B_xx + scatter_0) / (beta_0 a + 1),
    and after the second (eta = 0.1, statistics averaged and normalised by the averaged
    weight sum, the carried second moment taken about the first batch's mean)
        Sigma_xx = (beta_1 B_xx + C_xx / W^) / (beta_1 a + 1).
    A large prior B and a small cell make beta matter; a third of the weights are zero,
    so counting them in M, or dropping eta from beta, or normalising by N instead of W^,
    fails this test."""
    rng = np.random.default_rng(404)
    lo, size = np.array([0.25, 0.5, 0.0]), np.array([0.0625, 0.0625, 0.0625])
    b = np.array([0.5, 0.5, 2e-4, 3e-4, 4e-4])
    a = 0.8
    opts = orc.Opts(K=1, iters=1, eta=0.1, prior_a=a, prior_b=tuple(b), min_samples=16)
    mix = synth.initial_mixtures(lo[None, :], size[None, :], 1)
    st = orc.new_state(1, 1)
    batches = [_k1_cell(rng, 300, 0.33, lo, size), _k1_cell(rng, 220, 0.33, lo, size)]

    P0 = batches[0][3:6].T.astype(np.float64)
    w0 = batches[0][6].astype(np.float64)
    M0, W0 = int((w0 > 0).sum()), w0.sum()
    assert M0 < w0.size
    assert orc.fit(opts, np.array([0, w0.size]), batches[0], mix, st)[0] == 0
    mean0 = (w0[:, None] * P0).sum(0) / W0
    D0 = P0 - mean0
    scatter0 = (w0[:, None] * D0).T @ D0  # unnormalised
    beta0 = 1.0 / M0
    Sxx0 = (beta0 * np.diag(b[2:]) + scatter0 / W0) / (beta0 * a + 1.0)
    assert mix["pi"][0] == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(mix["mu_pos"], mean0, rtol=1e-13)
    assert np.allclose(_unpack(mix["cov"])[2:, 2:], Sxx0, rtol=1e-11, atol=0)
    assert st["sw"][0] == pytest.approx(W0, rel=1e-14) and st["step"][0] == 1

    eta = 0.1
    P1 = batches[1][3:6].T.astype(np.float64)
    w1 = batches[1][6].astype(np.float64)
    M1, W1 = int((w1 > 0).sum()), w1.sum()
    assert orc.fit(opts, np.array([0, w1.size]), batches[1], mix, st)[0] == 0
    D1 = P1 - mean0                       # about the mean the first batch produced
    hW = (1.0 - eta) * W0 + eta * W1
    hS0 = hW                              # K = 1: S0 = W in each batch
    hS1 = eta * (w1[:, None] * D1).sum(0)
    hS2 = (1.0 - eta) * scatter0 + eta * (w1[:, None] * D1).T @ D1
    C = hS2 - np.outer(hS1, hS1) / hS0
    beta1 = eta / M1
    Sxx1 = (beta1 * np.diag(b[2:]) + C / hW) / (beta1 * a + hS0 / hW)
    assert np.allclose(mix["mu_pos"], mean0 + hS1 / hS0, rtol=1e-13)
    assert np.allclose(_unpack(mix["cov"])[2:, 2:], Sxx1, rtol=1e-11, atol=0)
    assert st["sw"][0] == pytest.approx(hW, rel=1e-14) and st["step"][0] == 2
    # the same batch with beta from a wrong count would be visibly different
    wrong = (eta / w1.size * np.diag(b[2:]) + C / hW) / (eta / w1.size * a + 1.0)
    assert np.abs(wrong - Sxx1).max() > 1e-6 * np.abs(Sxx1).max()


def test_accurate_sigma_default_prior_is_one_over_positive_count(orc):
    """The accurate covariance update (Sec. 3.2) with the default prior strength: with
    eta = 1, beta = 1 / M, M the count of positive weights. For K = 1 the positional block
    is (B_xx / M + scatter about the new mean) / (a / M + 1) exactly."""
    rng = np.random.default_rng(405)
    lo, size = np.array([0.5, 0.0, 0.25]), np.array([0.0625, 0.0625, 0.0625])
    b = np.array([0.5, 0.5, 2e-4, 3e-4, 4e-4])
    a = 0.8
    smp = _k1_cell(rng, 260, 0.3, lo, size)
    mix = synth.initial_mixtures(lo[None, :], size[None, :], 1)
    st = orc.new_state(1, 1)
    opts = orc.Opts(K=1, iters=1, prior_a=a, prior_b=tuple(b), accurate_sigma=1)
    assert orc.fit(opts, np.array([0, smp.shape[1]]), smp, mix, st)[0] == 0
    P = smp[3:6].T.astype(np.float64)
    w = smp[6].astype(np.float64)
    M, W = int((w > 0).sum()), w.sum()
    assert M < w.size
    D = P - mix["mu_pos"]
    scatter = (w[:, None] * D).T @ D / W
    beta = 1.0 / M
    Sxx = (beta * np.diag(b[2:]) + scatter) / (beta * a + 1.0)
    assert np.allclose(_unpack(mix["cov"])[2:, 2:], Sxx, rtol=1e-11, atol=0)


def _duff_frame(mu):
    """Rows (t1, t2, mu) of the branchless orthonormal basis of Duff et al. (2017),
    written from the published formulas for this test."""
    s = 1.0 if mu[2] >= 0.0 else -1.0
    a = -1.0 / (s + mu[2])
    b = mu[0] * mu[1] * a
    return np.array([[1.0 + s * mu[0] ** 2 * a, s * b, -s * mu[0]],
                     [b, s + mu[1] ** 2 * a, -mu[1]],
                     [mu[0], mu[1], mu[2]]])


def test_estep_jacobian_responsibilities_divide_by_sinc(orc):
    """Reading A2: with estep_jacobian the E-step weighs component k by its solid-angle
    density, the tangent density divided by sinc |nu_k| (Sec. 3.1). Written out directly
    for K = 3 with scipy's Gaussian density and geodesic coordinates: the oracle's
    responsibilities, and through a fit its S0 = sum w r and its new positional means,
    agree to rounding. The same data under the tangent densities (the default) differ
    from it, so the test sees which branch ran."""
    K = 3
    rng = np.random.default_rng(406)
    n = 400
    lobes = _unit(np.array([[0.1, 0.2, 1.0], [0.9, -0.3, 0.2], [-0.4, 0.8, -0.5]]))
    lab = rng.integers(0, K, n)
    smp = np.zeros((7, n), dtype=np.float32)
    smp[0:3] = synth.sample_vmf(rng, lobes[lab], np.full(n, 1.5)).T   # broad: large |nu|
    smp[3:6] = rng.random((3, n))
    smp[6] = synth.draw_weights(rng, n)
    mix = synth.initial_mixtures(np.zeros((1, 3)), np.ones((1, 3)), K)
    mix["mu_dir"][:] = lobes.ravel()
    mix["pi"][:] = [0.5, 0.3, 0.2]
    covs = []
    for k in range(K):
        A = rng.normal(size=(5, 5)) * 0.2
        S = A @ A.T + np.diag([0.6, 0.5, 0.08, 0.09, 0.1])
        covs.append(S)
        mix["cov"][15 * k:15 * k + 15] = _pack(S)
    mus = mix["mu_pos"].reshape(K, 3)
    W = smp[6].astype(np.float64)

    def direct(jac):
        R = np.zeros((n, K))
        for i in range(n):
            om, p = smp[0:3, i].astype(np.float64), smp[3:6, i].astype(np.float64)
            dens = np.zeros(K)
            for k in range(K):
                v = _duff_frame(lobes[k]) @ om
                th = np.arctan2(np.hypot(v[0], v[1]), v[2])
                nu = th / np.hypot(v[0], v[1]) * v[:2]
                y = np.concatenate([nu, p - mus[k]])
                dens[k] = mix["pi"][k] * multivariate_normal(np.zeros(5), covs[k]).pdf(y)
                if jac:
                    r = np.linalg.norm(nu)
                    dens[k] /= np.sin(r) / r
            R[i] = dens / dens.sum()
        return R

    Rj, Rt = direct(True), direct(False)
    assert np.abs(Rj - Rt).max() > 1e-2
    oj = orc.Opts(K=K, estep_jacobian=1, prior_mode=1, prior_scale=0.0)
    for i in range(0, n, 9):
        r = orc.responsibilities(oj, smp[0:3, i], smp[3:6, i], mix)
        assert np.allclose(r, Rj[i], rtol=1e-11, atol=1e-14), (i, r, Rj[i])
    st = orc.new_state(1, K)
    m2 = synth.copy_mix(mix)
    assert orc.fit(oj, np.array([0, n]), smp, m2, st)[0] == 0
    S0 = (W[:, None] * Rj).sum(0)
    assert np.allclose(st["s0"], S0, rtol=1e-11)
    P = smp[3:6].T.astype(np.float64)
    newx = ((W[:, None] * Rj).T @ P) / S0[:, None]
    assert np.allclose(m2["mu_pos"].reshape(K, 3), newx, rtol=1e-11)


def test_openmp_build_gives_the_same_cells(orc):
    """The all-cores CPU baseline runs the same oracle source built with OpenMP over
    cells. Cells are independent, so the result is bitwise the single-threaded one."""
    wl = synth.workload("cells4k", scale=27 / 4096)
    b = synth.workload_batch(wl)
    C = wl["grid"].n_cells
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    m1, s1 = synth.copy_mix(mix0), orc.new_state(C, 16)
    m4, s4 = synth.copy_mix(mix0), orc.new_state(C, 16)
    st1 = orc.fit(orc.Opts(K=16, iters=2), b.offsets, b.samples, m1, s1)
    st4 = orc.fit(orc.Opts(K=16, iters=2), b.offsets, b.samples, m4, s4, threads=4)
    assert orc.threads_in_use(4) == 4
    assert np.array_equal(st1, st4)
    for k in m1:
        assert np.array_equal(m1[k], m4[k]), k
    for k in s1:
        assert np.array_equal(s1[k], s4[k]), k
