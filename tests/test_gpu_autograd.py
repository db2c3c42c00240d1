"""GPU tests of the autograd binding (paper_2111_13094_amd.autograd): gradients through
the parameter map, with a non-zero tangent offset delta and a negative Cholesky pivot,
against FP64 central differences of the oracle objective at the mixture that the oracle's
own exp map and products give; and gradient refinement of a fitted state.

Tolerance: each gradient block of a cell within 2e-4 of the block's largest magnitude,
the positional and directional mean blocks compared after whitening by L^T (the gradient
with respect to the mean in units of the component's own standard deviations), because
the device pass forms sample offsets in FP32."""
import numpy as np
import pytest

from paper_2111_13094_amd import synth
from tests.parity_utils import pack, to_torch

pytestmark = pytest.mark.gpu

TRI = [(d, e) for d in range(5) for e in range(d + 1)]


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_13094_amd import sdmm
    sdmm.lib()
    return torch


def _lower(l15):
    Lm = np.zeros((5, 5))
    for i, (d, e) in enumerate(TRI):
        Lm[d, e] = l15[i]
    return Lm


def _orc_cell_mixture(orc, alpha, mu0, delta, mu_pos, L):
    """One cell's mixture from the parameters with the oracle's exp map (FP64)."""
    K = alpha.size
    e = np.exp(alpha - alpha.max())
    mud = np.zeros((K, 3))
    cov = np.zeros((K, 15))
    for k in range(K):
        m0 = mu0[k] / np.linalg.norm(mu0[k])
        w = orc.exp_map(m0, delta[k])
        mud[k] = w / np.linalg.norm(w)
        Lm = _lower(L[k])
        cov[k] = pack(Lm @ Lm.T)
    return {"pi": e / e.sum(), "mu_dir": mud.ravel(), "mu_pos": mu_pos.ravel().copy(), "cov": cov.ravel()}


def _whiten(g_delta, g_mu_pos, L):
    """L^T [g_delta; g_mu_pos] per component."""
    out = np.zeros((g_delta.shape[0], 5))
    for k in range(g_delta.shape[0]):
        out[k] = _lower(L[k]).T @ np.concatenate([g_delta[k], g_mu_pos[k]])
    return out


def _problem(orc, seed=5):
    wl = synth.workload("cells4k", scale=8 / 4096, seed=seed)
    C = wl["grid"].n_cells
    b = synth.workload_batch(wl)
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    orc.fit(orc.Opts(K=16, iters=3), b.offsets, b.samples, mix, orc.new_state(C, 16))
    return wl, b, mix


def test_autograd_matches_finite_differences_of_the_oracle(dev, orc):
    print("case: autograd through the parameter map vs oracle FD (2 cells)", flush=True)
    from paper_2111_13094_amd import autograd, sdmm
    torch = dev
    wl, b, mix = _problem(orc)
    C, K = wl["grid"].n_cells, 16
    beta = 0.02
    opts = sdmm.default_opts(K, prior_mode=sdmm.PRIOR_FIXED, prior_scale=beta)
    p = autograd.params_from_mixture(to_torch(mix), C, K)
    rng = np.random.default_rng(2)
    with torch.no_grad():
        p["delta"].copy_(torch.from_numpy(0.05 * rng.normal(size=(C, K, 2))).cuda())
        p["alpha"].add_(torch.from_numpy(0.3 * rng.normal(size=(C, K))).cuda())
        p["L"][0, 3, 0] = -p["L"][0, 3, 0]  # a negative pivot: same Sigma, column sign flips
        p["L"][0, 3, 1:3] = -p["L"][0, 3, 1:3]
    off, smp = torch.from_numpy(b.offsets).cuda(), torch.from_numpy(b.samples).cuda()
    F, status = autograd.penalised_log_likelihood(p, off, smp, opts)
    assert (status.cpu().numpy() == 0).all()
    F.sum().backward()
    P = {k: v.detach().cpu().numpy() for k, v in p.items()}
    G = {k: p[k].grad.cpu().numpy() for k in ("alpha", "delta", "mu_pos", "L")}
    oo = orc.Opts(K=K, prior_mode=1, prior_scale=beta)
    for c in (0, 5):
        i0, i1 = b.offsets[c], b.offsets[c + 1]

        def f(q):
            m = _orc_cell_mixture(orc, q["alpha"], P["mu_dir0"][c], q["delta"], q["mu_pos"], q["L"])
            return orc.objective(oo, b.samples, i0, i1, m, beta, cell=0)

        base = {k: P[k][c].copy() for k in ("alpha", "delta", "mu_pos", "L")}
        assert abs(F[c].item() - f(base)) <= 1e-6 * abs(f(base))
        fd = {}
        for key, v in base.items():
            g = np.zeros_like(v)
            flat = v.reshape(-1)
            for j in range(flat.size):
                h = 1e-6 * max(abs(flat[j]), 1e-2)
                q = {k: x.copy() for k, x in base.items()}
                q[key].reshape(-1)[j] = flat[j] + h
                fp = f(q)
                q[key].reshape(-1)[j] = flat[j] - h
                g.reshape(-1)[j] = (fp - f(q)) / (2 * h)
            fd[key] = g
        errs = {key: np.abs(G[key][c] - fd[key]).max() / np.abs(fd[key]).max() for key in fd}
        wg = _whiten(G["delta"][c], G["mu_pos"][c], P["L"][c])
        wf = _whiten(fd["delta"], fd["mu_pos"], P["L"][c])
        errs["mean (whitened)"] = np.abs(wg - wf).max() / np.abs(wf).max()
        print(c, {k: "%.2e" % v for k, v in errs.items()})
        for key in ("alpha", "L", "mean (whitened)"):
            assert errs[key] < 2e-4, (c, key, errs)


def test_refinement_increases_the_objective(dev, orc):
    print("case: 10 refinement steps on 8 cells after 2 EM iterations", flush=True)
    from paper_2111_13094_amd import autograd, sdmm
    torch = dev
    wl = synth.workload("cells4k", scale=8 / 4096, seed=6)
    C, K = wl["grid"].n_cells, 16
    b = synth.workload_batch(wl)
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], K)
    orc.fit(orc.Opts(K=K, iters=2), b.offsets, b.samples, mix, orc.new_state(C, K))
    opts = sdmm.default_opts(K, prior_mode=sdmm.PRIOR_FIXED, prior_scale=1e-3)
    off, smp = torch.from_numpy(b.offsets).cuda(), torch.from_numpy(b.samples).cuda()
    refined, F0, F1, status = autograd.refine(to_torch(mix), C, K, off, smp, opts, steps=10, lr=1e-3)
    torch.cuda.synchronize()
    F0, F1 = F0.cpu().numpy(), F1.cpu().numpy()
    print("F before", F0, "after", F1)
    assert (status.cpu().numpy() == 0).all()
    assert (F1 > F0).all(), (F0, F1)
    # the refined mixture is a valid mixture: weights sum to 1, unit directions
    r = {k: v.cpu().numpy() for k, v in refined.items()}
    assert np.allclose(r["pi"].reshape(C, K).sum(1), 1.0, atol=1e-12)
    assert np.allclose(np.linalg.norm(r["mu_dir"].reshape(-1, 3), axis=1), 1.0, atol=1e-12)
