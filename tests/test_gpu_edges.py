"""GPU parity on the method's edge cases, through the C ABI, against the FP64 oracle.

The tangent log map of Sec. 3.1 has two special points per component: the mean itself
(theta = 0, where theta / sin theta -> 1) and the antipode (theta = pi, the cut locus, where
the map is singular; reading A15 sends it to (pi, 0) in the E-step, gives a pdf
contribution of 0 at |nu| >= pi (1 - 1e-6), and discards draws with |nu| >= pi). These
tests put samples, pdf directions and draws exactly there and next to them.

The component means are axis vectors. Their frames (Duff et al. 2017) have entries 0 and
+-1, so the FP32 rotation of a direction is exact and the tests see the log map's own
arithmetic; for a general mean the FP32 rotation of a near-antipodal direction carries an
absolute error of about 1e-7, which the 1 / sinc factor of the solid-angle density
multiplies by 1 / (pi - theta)."""
import numpy as np
import pytest

from paper_2111_13094_amd import synth
from tests.parity_utils import (CUT_LOCUS_BAND, assert_close, compare_mixtures, draw_radius, state_to_torch,
                                to_numpy, to_torch)

pytestmark = pytest.mark.gpu

K = 16
AXES = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1], [0, 0, 1], [0, -1, 0]],
                dtype=np.float64)


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_13094_amd import sdmm
    sdmm.lib()
    return torch


def _axis_mixture(rng, lo, size, broad=False):
    """K = 16 components: two spatial means crossed with eight axis directions. With
    broad, random SPD covariances with directional variances near 1 rad^2 and
    direction-position correlation, so that |nu| = pi is reachable by sampling."""
    mix = synth.initial_mixtures(lo[None, :], size[None, :], K)
    mud = mix["mu_dir"].reshape(K, 3)
    for k in range(K):
        mud[k] = AXES[k % 8]
    if broad:
        for k in range(K):
            A = rng.normal(size=(5, 5)) * np.array([0.5, 0.5, 0.05, 0.05, 0.05])[:, None]
            S = A @ A.T + np.diag([0.8, 0.7, 0.004, 0.005, 0.006])
            mix["cov"][15 * k:15 * k + 15] = [S[d, e] for d in range(5) for e in range(d + 1)]
        p = rng.dirichlet(np.full(K, 2.0))
        mix["pi"][:] = p
    return mix


def _tangent_point(mu, theta, phi):
    """The unit direction at angle theta from the axis vector mu, towards phi."""
    t1 = np.array([mu[1], mu[2], mu[0]])  # another axis, orthogonal to mu
    t2 = np.cross(mu, t1)
    return np.cos(theta) * mu + np.sin(theta) * (np.cos(phi) * t1 + np.sin(phi) * t2)


def _edge_cell(seed=61, n=4096):
    """One cell of n samples: half from the planted lobes, then in equal parts exactly at
    a component mean, exactly at its antipode, and at 1e-5 and 1e-3 rad from a mean
    (FP32 directions; positions and weights from the generator)."""
    wl = synth.workload("single", seed=seed)
    b = synth.make_batch(seed + 1, [n], wl["box_lo"], wl["box_size"], wl["lobes"], parallax=True)
    rng = np.random.default_rng(seed + 2)
    q = n // 8
    for part, (kind, theta) in enumerate((("at", 0.0), ("anti", 0.0), ("near", 1e-5), ("near", 1e-3))):
        for i in range(q):
            idx = n // 2 + part * q + i
            mu = AXES[(i + part) % 8]
            if kind == "at":
                d = mu
            elif kind == "anti":
                d = -mu
            else:
                d = _tangent_point(mu, theta, rng.uniform(0, 2 * np.pi))
            b.samples[0:3, idx] = d.astype(np.float32)
    return wl, b


@pytest.mark.parametrize("sched", ["batched", "fused"])
def test_fit_with_samples_at_means_and_antipodes(dev, orc, sched):
    """One E+M step on a cell whose samples include omega = mu_k, omega = -mu_k and
    omega at 1e-5 and 1e-3 rad from mu_k: element-wise parity with the oracle at the
    stated bar."""
    print(f"case: edge samples (mean, antipode, 1e-5, 1e-3 rad), one E+M step, {sched}", flush=True)
    from paper_2111_13094_amd import sdmm
    wl, b = _edge_cell()
    mix0 = _axis_mixture(np.random.default_rng(1), wl["box_lo"][0], wl["box_size"][0])
    om, ost = synth.copy_mix(mix0), orc.new_state(1, K)
    s_o = orc.fit(orc.Opts(K=K), b.offsets, b.samples, om, ost)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(1, K))
    o = sdmm.default_opts(K, schedule=sdmm.SCHED_FUSED if sched == "fused" else sdmm.SCHED_BATCHED)
    s_g = sdmm.fit_mixtures(dev.from_numpy(b.offsets).cuda(), dev.from_numpy(b.samples).cuda(), gm, gst, o)
    dev.cuda.synchronize()
    assert (s_g.cpu().numpy() == s_o).all(), (s_g, s_o)
    got = to_numpy(gm)
    for k in got:
        assert np.isfinite(got[k]).all(), k
    worst = compare_mixtures(got, om, K)
    print(worst)
    assert_close(worst, what=f"edge samples, {sched}")
    g = to_numpy(gst)
    assert np.allclose(g["s0"], ost["s0"], rtol=1e-4, atol=1e-7 * ost["sw"][0])


def _queries(rng, lo, size, nq):
    qpos = (lo + rng.random((nq, 3)) * size).astype(np.float32)
    return qpos, np.zeros(nq, dtype=np.int32)


def _gpu_cond(dev, mix, qpos, qcell):
    from paper_2111_13094_amd import sdmm
    table = sdmm.condition_prepare(to_torch(mix), 1, K)
    qp = dev.from_numpy(np.ascontiguousarray(qpos.T)).cuda()
    qc = dev.from_numpy(qcell).cuda()
    cw, cm = sdmm.condition(table, 1, K, qp, qc)
    return table, qp, qc, cw, cm


def _near_cut_threshold(mix, d):
    """True when some component's geodesic angle to d is within FP32 reach of the pdf's
    cut threshold pi (1 - 1e-6): both outcomes are correct there."""
    mud = mix["mu_dir"].reshape(K, 3)
    for mu in mud:
        th = np.arctan2(np.linalg.norm(np.cross(mu, d)), mu @ d)
        if abs(th - np.pi * (1.0 - 1e-6)) < 3e-7 * np.pi:
            return True
    return False


def test_pdf_at_means_and_near_the_cut_locus(dev, orc):
    """The conditioned pdf at directions exactly at a component mean, at 1e-5 and 1e-3
    rad from it, exactly at its antipode, and at pi - eps with eps / pi in
    {2e-7, 5e-7} (inside the zero band |nu| >= pi (1 - 1e-6)) and {2e-6, 5e-6, 1e-5, 1e-4}
    (outside it, where 1 / sinc |nu| reaches 5e5): relative 1e-4 against the oracle
    wherever the pdf exceeds 1e-6 of the query's largest value."""
    print("case: pdf at means, antipodes and |nu| near pi", flush=True)
    from paper_2111_13094_amd import sdmm
    rng = np.random.default_rng(71)
    lo, size = np.array([0.25, 0.5, 0.0]), np.array([0.0625, 0.0625, 0.0625])
    mix = _axis_mixture(rng, lo, size, broad=True)
    nq = 8
    qpos, qcell = _queries(rng, lo, size, nq)
    thetas = [0.0, 1e-5, 1e-3] + [np.pi * (1.0 - e) for e in (0.0, 2e-7, 5e-7, 2e-6, 5e-6, 1e-5, 1e-4)]
    dirs = []
    for mu in AXES[:6]:
        for th in thetas:
            dirs.append(_tangent_point(mu, th, rng.uniform(0, 2 * np.pi)))
    dirs = np.array(dirs, dtype=np.float32)
    nd = dirs.shape[0]
    d = np.tile(dirs[None], (nq, 1, 1))
    table, qp, qc, cw, cm = _gpu_cond(dev, mix, qpos, qcell)
    gd = dev.from_numpy(np.ascontiguousarray(d.reshape(-1, 3).T)).cuda()
    got = sdmm.pdf(table, 1, K, qc, cw, cm, gd, nd).cpu().numpy().reshape(nq, nd)
    ref = orc.pdf(K, mix, qpos.astype(np.float64), qcell, d.astype(np.float64))
    assert np.isfinite(got).all()
    worst = 0.0
    checked = 0
    for q in range(nq):
        for t in range(nd):
            if _near_cut_threshold(mix, d[q, t].astype(np.float64)):
                continue
            if ref[q, t] > 1e-6 * ref[q].max():
                rel = abs(got[q, t] - ref[q, t]) / ref[q, t]
                worst = max(worst, rel)
                assert rel < 1e-4, (q, t, got[q, t], ref[q, t])
                checked += 1
            else:
                assert abs(got[q, t]) <= 2e-6 * ref[q].max(), (q, t, got[q, t], ref[q, t])
    print("pdf worst relative %.2e over %d values" % (worst, checked))
    assert checked > nq * nd // 2


def _uniforms_for_radius(rng, pic, m, Sc, k, radius):
    """Uniforms (u0, u1, u2) that select component k (middle of its CDF interval) and
    draw nu = m_k + chol(Sc_k) z at |nu| = radius, by inverting Box-Muller; None when
    that needs u1 within FP32 rounding of 1."""
    cdf = np.concatenate([[0.0], np.cumsum(pic)])
    u0 = 0.5 * (cdf[k] + cdf[k + 1])
    L = np.linalg.cholesky(np.array([[Sc[k, 0], Sc[k, 1]], [Sc[k, 1], Sc[k, 2]]]))
    phi = rng.uniform(0, 2 * np.pi)
    nu = radius * np.array([np.cos(phi), np.sin(phi)])
    z = np.linalg.solve(L, nu - m[k])
    r2 = z @ z
    if r2 > 28.0:
        return None
    u1 = -np.expm1(-0.5 * r2)
    u2 = (np.arctan2(z[1], z[0]) / (2 * np.pi)) % 1.0
    u = np.array([u0, u1, u2], dtype=np.float32)
    if not (u < 1.0).all():
        return None
    return u


def test_sampling_at_the_cut_locus(dev, orc):
    """Draws aimed at |nu| = pi (1 + delta) for delta from -1e-4 to 1e-4 (caller
    uniforms built by inverting Box-Muller). Wherever the FP64 radius of the draw, from
    the same FP32 uniforms, is farther than 1e-5 from pi, the device and the oracle agree
    on its validity (discard at |nu| >= pi); valid draws agree in direction (1e-5 rad);
    and the returned pdf equals the oracle's pdf at the returned direction (relative
    1e-4), the property a renderer relies on, since near the antipode the pdf changes by
    1 / (pi - |nu|) per radian of direction. The separate and fused calls agree."""
    print("case: sampling with |nu| near pi", flush=True)
    from paper_2111_13094_amd import sdmm
    rng = np.random.default_rng(81)
    lo, size = np.array([0.5, 0.25, 0.75]), np.array([0.0625, 0.0625, 0.0625])
    mix = _axis_mixture(rng, lo, size, broad=True)
    nq = 16
    qpos, qcell = _queries(rng, lo, size, nq)
    deltas = [-1e-4, -1e-5, -3e-6, -1e-6, 0.0, 1e-6, 3e-6, 1e-5, 1e-4]
    ns = len(deltas) + 3
    u = np.zeros((nq, ns, 3), dtype=np.float32)
    for q in range(nq):
        pic, m, Sc = orc.condition(K, mix, 0, qpos[q].astype(np.float64))
        heavy = np.nonzero(pic > 1e-3)[0]
        for t in range(ns):
            uu = None
            tries = 0
            while uu is None:
                k = heavy[rng.integers(0, heavy.size)]
                if t < len(deltas):
                    uu = _uniforms_for_radius(rng, pic, m, Sc, k, np.pi * (1.0 + deltas[t]))
                else:  # ordinary draws
                    uu = rng.random(3, dtype=np.float32)
                tries += 1
                assert tries < 100
            u[q, t] = uu
    table, qp, qc, cw, cm = _gpu_cond(dev, mix, qpos, qcell)
    gu = dev.from_numpy(np.ascontiguousarray(u.reshape(-1, 3).T)).cuda()
    dirs, pdfv, valid, comp = sdmm.sample(table, 1, K, qc, cw, cm, ns, uniforms=gu, with_comp=True)
    gd = dirs.cpu().numpy().T.reshape(nq, ns, 3)
    gp = pdfv.cpu().numpy().reshape(nq, ns)
    gv = valid.cpu().numpy().reshape(nq, ns)
    gc = comp.cpu().numpy().reshape(nq, ns)
    od, op, oc, ov = orc.sample(K, mix, qpos.astype(np.float64), qcell, u.astype(np.float64))
    at_pdf = orc.pdf(K, mix, qpos.astype(np.float64), qcell, gd.astype(np.float64))
    decided = near = 0
    for q in range(nq):
        pic, m, Sc = orc.condition(K, mix, 0, qpos[q].astype(np.float64))
        for t in range(ns):
            assert gc[q, t] == oc[q, t], (q, t, gc[q, t], oc[q, t])
            r = draw_radius(m[oc[q, t]], Sc[oc[q, t]], u[q, t].astype(np.float64))
            if abs(r - np.pi) < CUT_LOCUS_BAND:
                near += 1
            else:
                decided += 1
                assert gv[q, t] == ov[q, t], (q, t, r, gv[q, t], ov[q, t])
            if not gv[q, t]:
                assert np.all(gd[q, t] == 0) and gp[q, t] == 0
                continue
            if ov[q, t]:
                a, b = gd[q, t].astype(np.float64), od[q, t]
                ang = np.arctan2(np.linalg.norm(np.cross(a, b)), a @ b)
                assert ang < 1e-5, (q, t, ang)
            if not _near_cut_threshold(mix, gd[q, t].astype(np.float64)):
                assert abs(gp[q, t] - at_pdf[q, t]) <= 1e-4 * at_pdf[q, t], (q, t, gp[q, t], at_pdf[q, t])
    print("draws decided %d, within the band %d, invalid %d" % (decided, near, int((ov == 0).sum())))
    assert decided >= nq * 6 and (ov == 0).sum() >= nq * 3
    fd, fp, fv = sdmm.condition_sample_pdf(table, 1, K, qp, qc, ns, uniforms=gu)
    assert dev.equal(fv, valid)
    assert np.allclose(fd.cpu().numpy(), dirs.cpu().numpy(), rtol=0, atol=1e-6)
    assert np.allclose(fp.cpu().numpy(), pdfv.cpu().numpy(), rtol=1e-6, atol=0)
