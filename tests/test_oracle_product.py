"""Pins for the oracle's product sampling with a conditioned BSDF mixture (Sec. 3.4, and
the pruning to two BSDF components of Sec. 4.1). Independent references: central
differences of the composed maps, rotation invariance of the density, grid quadrature of
the product of two Gaussians, sphere quadrature, a chi-square test of the draws, and the
exact product of the two conditioned densities on the sphere."""
import numpy as np
import pytest
from scipy.stats import chisquare, multivariate_normal

from paper_2111_13094_amd import synth


def _unit(v):
    return v / np.linalg.norm(v)


def _fd_jacobian(f, x, h=1e-6):
    x = np.asarray(x, dtype=float)
    cols = []
    for j in range(x.size):
        e = np.zeros_like(x)
        e[j] = h
        cols.append((f(x + e) - f(x - e)) / (2 * h))
    return np.stack(cols, axis=1)


def _fitted(orc, iters=3, n=4096, seed=5, K=16):
    wl = synth.workload("single", seed=seed)
    b = synth.make_batch(seed + 1, [n], wl["box_lo"], wl["box_size"], wl["lobes"], parallax=True)
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], K)
    orc.fit(orc.Opts(K=K, iters=iters), b.offsets, b.samples, mix, orc.new_state(1, K))
    return mix


def _sphere_grid(nt, nphi):
    th = (np.arange(nt) + 0.5) * np.pi / nt
    ph = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    T, P = np.meshgrid(th, ph, indexing="ij")
    dirs = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(-1, 3)
    wts = (np.sin(T) * (np.pi / nt) * (2 * np.pi / nphi)).ravel()
    return dirs, wts


def _S2(c):
    return np.array([[c[0], c[1]], [c[1], c[2]]])


def _query(seed=3):
    bpar, bcell, F = synth.bsdf_queries(seed, 1)
    return np.array([0.45, 0.55, 0.5]), bpar[0], F[0]


# --- pair transfer -------------------------------------------------------------------

def test_pair_transfer_matches_finite_differences(orc):
    """a = log_mu1(exp_mu2(m2)) and J = d(log_mu1 o exp_mu2)/d nu at m2, against the maps
    and central differences of the composed maps."""
    rng = np.random.default_rng(11)
    for _ in range(40):
        mu2 = _unit(rng.normal(size=3))
        mu1 = _unit(mu2 + rng.uniform(0.0, 1.5) * rng.normal(size=3))
        m2 = rng.normal(size=2) * rng.choice([0.0, 1e-3, 0.2, 0.8])
        a, J = orc.pair_transfer(mu1, mu2, m2)
        f = lambda v: orc.log_map(mu1, orc.exp_map(mu2, v))
        assert np.allclose(a, f(m2), atol=1e-14)
        assert np.allclose(J, _fd_jacobian(f, m2), atol=2e-8), (mu1, mu2, m2)


def test_pair_transfer_near_the_mean_uses_the_limit(orc):
    """When the centre lands on mu1 (s -> 0) the log-map Jacobian takes its limit."""
    rng = np.random.default_rng(12)
    for _ in range(10):
        mu2 = _unit(rng.normal(size=3))
        m2 = 0.3 * rng.normal(size=2)
        mu1 = orc.exp_map(mu2, m2)
        mu1 = mu1 / np.linalg.norm(mu1)
        a, J = orc.pair_transfer(mu1, mu2, m2)
        assert np.abs(a).max() < 1e-12
        f = lambda v: orc.log_map(mu1, orc.exp_map(mu2, v))
        assert np.allclose(J, _fd_jacobian(f, m2), atol=2e-8)
        # the same map as the M-step's first-order transfer, by a separate code path
        assert np.allclose(J, orc.transfer_jacobian(mu2, m2), atol=1e-12)


# --- rotation to world -----------------------------------------------------------------

def test_rotation_to_world_is_exact(orc):
    """The rotated component's density at F w equals the local component's density at w."""
    rng = np.random.default_rng(13)
    for F in synth.random_rotations(rng, 20):
        mu = _unit(rng.normal(size=3))
        m = 0.3 * rng.normal(size=2)
        Lm = np.tril(rng.normal(size=(2, 2))) * 0.3 + np.diag([0.2, 0.2])
        S2 = Lm @ Lm.T
        S = np.array([S2[0, 0], S2[1, 0], S2[1, 1]])
        muw, mw, Sw = orc.rotate_component(F, mu, m, S)
        assert np.allclose(muw, F @ mu, atol=1e-15)
        for w in [_unit(rng.normal(size=3)) for _ in range(5)]:
            pl = orc.pdf_conditioned(1, mu, [1.0], m, S, w)
            pw = orc.pdf_conditioned(1, muw, [1.0], mw, Sw, F @ w)
            if pl == 0.0:  # beyond the cut locus
                assert pw == 0.0
                continue
            # far in the tail the density is exp(-q/2) with q in the hundreds, so compare
            # the logarithms, to the relative rounding of q
            assert np.log(pw) == pytest.approx(np.log(pl), rel=1e-11, abs=1e-12)


# --- the product of two Gaussians ------------------------------------------------------

def test_pair_product_by_grid_quadrature(orc):
    """With the BSDF component rotated onto the radiance component's mean, the transfer
    is the identity, and each pair must be the product of the two tangent Gaussians:
    weight pi' w times its integral, mean and covariance its normalised moments, all by
    quadrature on a grid."""
    K, Kb = 1, 1
    mix = synth.initial_mixtures(np.zeros((1, 3)), np.ones((1, 3)), K)
    mix["cov"][0] = 0.3
    mix["cov"][2] = 0.2
    mix["cov"][1] = 0.05
    mix["cov"][3 + 0] = 0.02  # direction-position coupling (row 2, col 0)
    bmix = synth.bsdf_mixtures(4, 1, Kb)
    x, bx = np.array([0.6, 0.4, 0.55]), np.array([0.7, 3.0, 0.3])
    # choose F so that F mu_b = mu_k
    mu_k = mix["mu_dir"][:3]
    mu_b = bmix["mu_dir"][:3]
    v = np.cross(mu_b, mu_k)
    c, s = mu_b @ mu_k, np.linalg.norm(v)
    vx = np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]])
    F = np.eye(3) + vx + vx @ vx * ((1 - c) / s ** 2)
    assert np.allclose(F @ mu_b, mu_k, atol=1e-14)
    pr = orc.product_pairs(K, mix, 0, Kb, bmix, 0, x, bx, F)
    pic, m, Sc = orc.condition(K, mix, 0, x)
    bpic, bm, bSc = orc.condition(Kb, bmix, 0, bx)
    muw, mw, Sw = orc.rotate_component(F, mu_b, bm[0], bSc[0])
    a, J = orc.pair_transfer(mu_k, muw, mw)
    assert np.allclose(J, np.eye(2), atol=1e-12) and np.allclose(a, mw, atol=1e-12)
    A, B = _S2(Sc[0]), _S2(Sw)
    sd = np.sqrt(max(np.diag(A).max(), np.diag(B).max()))
    ctr = 0.5 * (m[0] + mw)
    g0 = np.linspace(ctr[0] - 12 * sd, ctr[0] + 12 * sd, 1201)
    g1 = np.linspace(ctr[1] - 12 * sd, ctr[1] + 12 * sd, 1201)
    G0, G1 = np.meshgrid(g0, g1, indexing="ij")
    Y = np.stack([G0.ravel(), G1.ravel()], 1)
    p = multivariate_normal(m[0], A).pdf(Y) * multivariate_normal(mw, B).pdf(Y)
    area = (g0[1] - g0[0]) * (g1[1] - g1[0])
    Z = p.sum() * area
    mean = (p[:, None] * Y).sum(0) * area / Z
    D = Y - mean
    cov = (p[:, None] * D).T @ D * area / Z
    assert np.exp(pr["logw"][0]) == pytest.approx(pic[0] * bpic[0] * Z, rel=1e-8)
    assert np.allclose(pr["c"][0], mean, atol=1e-9)
    assert np.allclose(_S2(pr["C"][0]), cov, rtol=1e-7, atol=1e-12)
    assert pr["logw"][1] == -np.inf  # one BSDF component: the second pair is empty


# --- pruning -----------------------------------------------------------------------------

def test_pruning_keeps_the_two_heaviest_bsdf_components(orc):
    """Only the two BSDF components of largest conditioned weight enter the product:
    changing any other component's shape leaves the density unchanged; on a tie the
    lower index wins."""
    K, Kb = 16, 6
    mix = _fitted(orc)
    bmix = synth.bsdf_mixtures(5, 1, Kb)
    x, bx, F = _query()
    bpic, _, _ = orc.condition(Kb, bmix, 0, bx)
    order = np.argsort(-bpic, kind="stable")
    rng = np.random.default_rng(2)
    dirs = np.stack([_unit(rng.normal(size=3)) for _ in range(64)])[None]
    p0 = orc.product_pdf(K, mix, Kb, bmix, x[None], [0], bx[None], [0], F[None], dirs)
    b2 = synth.copy_mix(bmix)
    for b in order[2:]:  # move the light components' directions and widths
        b2["mu_dir"][3 * b:3 * b + 3] = _unit(rng.normal(size=3))
        b2["cov"][15 * b] *= 2.0
    assert np.array_equal(orc.product_pdf(K, mix, Kb, b2, x[None], [0], bx[None], [0], F[None], dirs), p0)
    b3 = synth.copy_mix(bmix)
    b3["mu_dir"][3 * order[1]:3 * order[1] + 3] = _unit(rng.normal(size=3))
    assert not np.allclose(orc.product_pdf(K, mix, Kb, b3, x[None], [0], bx[None], [0], F[None], dirs), p0)
    # a tie: two identical components; the product keeps the lower index first
    b4 = synth.copy_mix(bmix)
    for key, n in (("pi", 1), ("mu_dir", 3), ("mu_pos", 3), ("cov", 15)):
        b4[key][n * 4:n * 5] = b4[key][n * order[0]:n * (order[0] + 1)]
    pr = orc.product_pairs(K, mix, 0, Kb, b4, 0, x, bx, F)
    lo = min(4, order[0])
    pr_ref = orc.product_pairs(K, mix, 0, Kb, bmix, 0, x, bx, F)
    # both kept pairs of component 0 now come from the tied pair, so they are equal
    assert pr["logw"][0] == pr["logw"][1]
    assert lo == min(4, order[0]) and np.isfinite(pr_ref["logw"][0])


# --- the product density -----------------------------------------------------------------

def _tail(c, C, n=401):
    sd = np.sqrt(np.diag(C)).max()
    half = np.pi + np.abs(c).max() + 12 * sd
    g = np.linspace(-half, half, n)
    G0, G1 = np.meshgrid(g, g, indexing="ij")
    Y = np.stack([G0.ravel(), G1.ravel()], 1)
    p = multivariate_normal(c, C).pdf(Y) * (g[1] - g[0]) ** 2
    return p[np.linalg.norm(Y, axis=1) >= np.pi].sum()


def test_product_pdf_integrates_to_one_minus_tail_mass(orc):
    K, Kb = 16, 8
    mix = _fitted(orc)
    bmix = synth.bsdf_mixtures(6, 1, Kb)
    x, bx, F = _query(7)
    pr = orc.product_pairs(K, mix, 0, Kb, bmix, 0, x, bx, F)
    P = np.exp(pr["logw"] - pr["logw"].max())
    P /= P.sum()
    tau = sum(P[p] * _tail(pr["c"][p], _S2(pr["C"][p])) for p in range(2 * K) if P[p] > 0)
    dirs, wts = _sphere_grid(1000, 2000)
    q = orc.product_pdf(K, mix, Kb, bmix, x[None], [0], bx[None], [0], F[None], dirs[None])[0]
    assert (q * wts).sum() == pytest.approx(1.0 - tau, abs=2e-6)


def test_product_sampling_matches_the_product_pdf(orc):
    K, Kb = 16, 8
    mix = _fitted(orc)
    bmix = synth.bsdf_mixtures(6, 1, Kb)
    x, bx, F = _query(9)
    n = 200000
    u = np.random.default_rng(19).random((1, n, 3))
    dirs, pdfv, pair, valid = orc.product_sample(K, mix, Kb, bmix, x[None], [0], bx[None], [0], F[None], u)
    dirs, pdfv, valid = dirs[0], pdfv[0], valid[0].astype(bool)
    again = orc.product_pdf(K, mix, Kb, bmix, x[None], [0], bx[None], [0], F[None], dirs[valid][None])[0]
    assert np.array_equal(again, pdfv[valid])
    assert np.all(pdfv[~valid] == 0) and np.all(dirs[~valid] == 0)
    nz, nph = 12, 12
    zb = np.clip(((dirs[valid, 2] + 1) / 2 * nz).astype(int), 0, nz - 1)
    pb = (np.mod(np.arctan2(dirs[valid, 1], dirs[valid, 0]), 2 * np.pi) / (2 * np.pi) * nph).astype(int) % nph
    obs = np.bincount(zb * nph + pb, minlength=nz * nph)
    qdirs, qw = _sphere_grid(720, 1440)
    qp = orc.product_pdf(K, mix, Kb, bmix, x[None], [0], bx[None], [0], F[None], qdirs[None])[0] * qw
    qz = np.clip(((qdirs[:, 2] + 1) / 2 * nz).astype(int), 0, nz - 1)
    qph = (np.mod(np.arctan2(qdirs[:, 1], qdirs[:, 0]), 2 * np.pi) / (2 * np.pi) * nph).astype(int) % nph
    exp = np.bincount(qz * nph + qph, weights=qp, minlength=nz * nph)
    keep = exp / exp.sum() * obs.sum() > 20
    stat = chisquare(obs[keep], exp[keep] * obs[keep].sum() / exp[keep].sum())
    assert stat.pvalue > 1e-4, stat


@pytest.mark.parametrize("scale", [1.0, 0.25])
def test_product_approximates_the_exact_product_of_densities(orc, scale):
    """The product mixture against the exact product of the conditioned radiance density
    and the conditioned, pruned BSDF density on the sphere (both normalised by
    quadrature): the first-order transfer makes it an approximation whose error shrinks
    as the BSDF lobes narrow."""
    K, Kb = 16, 6
    mix = _fitted(orc)
    bmix = synth.bsdf_mixtures(8, 1, Kb)
    bmix["cov"] *= scale ** 2
    x, bx, F = _query(4)
    dirs, wts = _sphere_grid(600, 1200)
    q = orc.product_pdf(K, mix, Kb, bmix, x[None], [0], bx[None], [0], F[None], dirs[None])[0]
    pR = orc.pdf(K, mix, x[None], [0], dirs[None])[0]
    bpic, bm, bSc = orc.condition(Kb, bmix, 0, bx)
    top = np.argsort(-bpic, kind="stable")[:2]
    pB = np.zeros(dirs.shape[0])
    for b in top:
        # the rotated component's solid-angle density, written out: geodesic tangent
        # coordinates in the frame of its mean, a 2-D Gaussian, divided by sinc
        muw, mw, Sw = orc.rotate_component(F, bmix["mu_dir"][3 * b:3 * b + 3], bm[b], bSc[b])
        p = dirs @ orc.frame(muw).T
        s = np.hypot(p[:, 0], p[:, 1])
        th = np.arctan2(s, p[:, 2])
        nu = (th / s)[:, None] * p[:, :2]
        dens = multivariate_normal(mw, _S2(Sw)).pdf(nu) * th / np.sin(th)
        pB += bpic[b] * np.where(th < np.pi * (1 - 1e-6), dens, 0.0)
    exact = pR * pB
    exact /= (exact * wts).sum()
    qn = q / (q * wts).sum()
    tv = 0.5 * (np.abs(qn - exact) * wts).sum()
    print(f"scale {scale}: total variation {tv:.3e}")
    assert tv < {1.0: 0.03, 0.25: 0.012}[scale], tv
