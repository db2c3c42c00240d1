"""Pins for the oracle's gradient of the penalised log-likelihood (the objective whose
maximiser is the MAP update of Sec. 4.3) and for planted-mixture recovery."""
import numpy as np
import pytest

from paper_2111_13094_amd import synth


def _tri(d, e):
    return d * (d + 1) // 2 + e


def _unpack_L(c):
    L = np.zeros((5, 5))
    for d in range(5):
        for e in range(d + 1):
            L[d, e] = c[_tri(d, e)]
    return L


def _pack(S):
    return np.array([S[d, e] for d in range(5) for e in range(d + 1)])


def _problem(orc, K=4, n=600, seed=9, euclid=False):
    wl = synth.workload("single", seed=seed)
    b = synth.make_batch(seed + 2, [n], wl["box_lo"], wl["box_size"], wl["lobes"], parallax=True)
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], K)
    opts = orc.Opts(K=K, iters=3, euclidean=int(euclid))
    st = orc.new_state(1, K)
    orc.fit(opts, b.offsets, b.samples, mix, st)
    rng = np.random.default_rng(seed)
    mix["pi"] = rng.dirichlet(np.ones(K) * 3)  # move off the fixed point
    return b, mix


@pytest.mark.parametrize("euclid", [False, True])
def test_gradient_matches_central_differences(orc, euclid):
    K = 4
    b, mix = _problem(orc, K=K, euclid=euclid)
    n = b.samples.shape[1]
    beta = 0.05
    opts = orc.Opts(K=K, prior_mode=1, prior_scale=beta, euclidean=int(euclid))
    g = orc.grad(opts, b.samples, 0, n, mix, beta)
    F = lambda m: orc.objective(opts, b.samples, 0, n, m, beta)
    h = 1e-6
    alpha = np.log(mix["pi"])

    def with_alpha(a):
        m = synth.copy_mix(mix)
        e = np.exp(a - a.max())
        m["pi"] = e / e.sum()
        return m

    for k in range(K):
        e = np.zeros(K)
        e[k] = h
        fd = (F(with_alpha(alpha + e)) - F(with_alpha(alpha - e))) / (2 * h)
        assert fd == pytest.approx(g["alpha"][k], rel=1e-6, abs=1e-7)
    for k in range(K):
        for d in range(3):
            mp, mm = synth.copy_mix(mix), synth.copy_mix(mix)
            mp["mu_pos"][3 * k + d] += h
            mm["mu_pos"][3 * k + d] -= h
            fd = (F(mp) - F(mm)) / (2 * h)
            assert fd == pytest.approx(g["mu_pos"][k, d], rel=1e-6, abs=1e-6)
    for k in range(K):
        mu = mix["mu_dir"][3 * k:3 * k + 3].copy()
        for j in range(2):
            dl = np.zeros(2)
            dl[j] = h
            mp, mm = synth.copy_mix(mix), synth.copy_mix(mix)
            if euclid:
                mp["mu_dir"][3 * k + j] += h
                mm["mu_dir"][3 * k + j] -= h
            else:
                wp, wm = orc.exp_map(mu, dl), orc.exp_map(mu, -dl)
                mp["mu_dir"][3 * k:3 * k + 3] = wp / np.linalg.norm(wp)
                mm["mu_dir"][3 * k:3 * k + 3] = wm / np.linalg.norm(wm)
            fd = (F(mp) - F(mm)) / (2 * h)
            assert fd == pytest.approx(g["delta"][k, j], rel=1e-5, abs=1e-6), (k, j)
    for k in range(K):
        L = np.linalg.cholesky(np.array(
            [[mix["cov"][15 * k + _tri(max(a, c), min(a, c))] for c in range(5)] for a in range(5)]))
        Lp = _pack(L)
        for t in range(15):
            lp, lm = Lp.copy(), Lp.copy()
            lp[t] += h
            lm[t] -= h
            mp, mm = synth.copy_mix(mix), synth.copy_mix(mix)
            Up, Um = _unpack_L(lp), _unpack_L(lm)
            mp["cov"][15 * k:15 * k + 15] = _pack(Up @ Up.T)
            mm["cov"][15 * k:15 * k + 15] = _pack(Um @ Um.T)
            fd = (F(mp) - F(mm)) / (2 * h)
            assert fd == pytest.approx(g["L"][k, t], rel=1e-5, abs=1e-5 * max(1.0, np.abs(g["L"][k]).max()))


def test_planted_lobes_are_recovered(orc):
    """Six well-separated planted vMF lobes (kappa 50-200, >= 60 degrees apart), unit
    weights, no parallax, no prior: the fitted directional marginal is close to the
    planted directional density in total variation and every lobe direction carries
    its planted mass. The marginal is obtained by conditioning a copy of the fit whose
    spatial blocks are identical and uncorrelated with the direction (then pi' = pi,
    m = 0 and Sigma' = Sigma_nn)."""
    lobes = synth.planted_lobes(77, min_sep_deg=60.0, kappa_range=(50.0, 200.0))
    b = synth.make_batch(78, [16384], np.zeros((1, 3)), np.ones((1, 3)), lobes, parallax=False,
                         weight_sigma=0.0, zero_frac=0.0)
    mix = synth.initial_mixtures(np.zeros((1, 3)), np.ones((1, 3)), 16)
    opts = orc.Opts(K=16, iters=60, prior_mode=1, prior_scale=0.0)
    st = orc.new_state(1, 16)
    orc.fit(opts, b.offsets, b.samples, mix, st)
    th = (np.arange(600) + 0.5) * np.pi / 600
    ph = (np.arange(1200) + 0.5) * 2 * np.pi / 1200
    T, P = np.meshgrid(th, ph, indexing="ij")
    dirs = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(-1, 3)
    wts = (np.sin(T) * (np.pi / 600) * (2 * np.pi / 1200)).ravel()
    marg = synth.copy_mix(mix)
    cov = marg["cov"].reshape(16, 15)
    for d in range(2, 5):
        for e in range(d + 1):
            cov[:, _tri(d, e)] = 1.0 if d == e else 0.0
    marg["mu_pos"][:] = 0.0
    x = np.array([0.5, 0.5, 0.5])
    p = orc.pdf(16, marg, x[None], np.array([0]), dirs[None])[0]
    planted = np.zeros(dirs.shape[0])
    for j in range(6):
        k = lobes.kappa[j]
        planted += lobes.weight[j] * k / (2 * np.pi * (1 - np.exp(-2 * k))) * np.exp(k * (dirs @ lobes.dirs[j] - 1))
    tv = 0.5 * (np.abs(p - planted) * wts).sum()
    assert tv < 0.05, tv
    mus = mix["mu_dir"].reshape(16, 3)
    for j in range(6):
        ang = np.arccos(np.clip(mus @ lobes.dirs[j], -1, 1))
        near = ang < 3.0 / np.sqrt(lobes.kappa[j])
        assert mix["pi"][near].sum() > 0.8 * lobes.weight[j], (j, mix["pi"][near].sum(), lobes.weight[j])
        mean_dir = (mix["pi"][near, None] * mus[near]).sum(0)
        mean_dir /= np.linalg.norm(mean_dir)
        assert np.arccos(np.clip(mean_dir @ lobes.dirs[j], -1, 1)) < 0.05
