"""GPU parity of the adjoint (sdmm_fit_grad through the C ABI) against the oracle's
objective and closed-form gradient, plus the stationarity check it is used for.

Tolerances: F relative 1e-6; each gradient block within 1e-4 of the block's largest
magnitude (the device pass accumulates FP32 products with compensated sums)."""
import numpy as np
import pytest

from paper_2111_13094_amd import synth
from tests.parity_utils import to_torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_13094_amd import sdmm
    sdmm.lib()
    return torch


def _problem(orc, seed=3, n_cells=27, iters=3, perturb=True):
    wl = synth.workload("cells4k", scale=n_cells / 4096, seed=seed)
    C = wl["grid"].n_cells
    b = synth.workload_batch(wl)
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    orc.fit(orc.Opts(K=16, iters=iters), b.offsets, b.samples, mix, orc.new_state(C, 16))
    if perturb:
        rng = np.random.default_rng(seed)
        pi = mix["pi"].reshape(C, 16) * np.exp(0.3 * rng.normal(size=(C, 16)))
        mix["pi"] = (pi / pi.sum(1, keepdims=True)).ravel()
    return wl, b, mix


def test_gradient_parity(dev, orc):
    print("case: adjoint on 27 cells", flush=True)
    from paper_2111_13094_amd import sdmm
    wl, b, mix = _problem(orc)
    C = wl["grid"].n_cells
    beta = 0.02
    o = sdmm.default_opts(16, prior_mode=sdmm.PRIOR_FIXED, prior_scale=beta)
    out = sdmm.fit_grad(dev.from_numpy(b.offsets).cuda(), dev.from_numpy(b.samples).cuda(), to_torch(mix), o)
    dev.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    assert (got["status"] == 0).all()
    oo = orc.Opts(K=16, prior_mode=1, prior_scale=beta)
    for c in range(C):
        i0, i1 = b.offsets[c], b.offsets[c + 1]
        F = orc.objective(oo, b.samples, i0, i1, mix, beta, cell=c)
        g = orc.grad(oo, b.samples, i0, i1, mix, beta, cell=c)
        assert abs(got["F"][c] - F) <= 1e-6 * abs(F), (c, got["F"][c], F)
        for key in ("alpha", "mu_pos", "delta", "L"):
            ref = g[key].reshape(16, -1)
            gg = got[key][c].reshape(16, -1)
            err = np.abs(gg - ref).max() / np.abs(ref).max()
            assert err < 1e-4, (c, key, err, np.abs(ref).max())


def test_gradient_vanishes_at_a_batch_em_fixed_point(dev, orc):
    """At a fixed point of batch MAP-EM (mean offsets m = 0, so the transfer Jacobian is
    the identity) the updates of the weights, positional means and covariances are exact
    maximisers of F, so those gradient blocks vanish up to the FP32 resolution of the
    pass; they are compared with the same blocks one EM step earlier on the way in."""
    print("case: stationarity after 400 EM iterations (8 cells)", flush=True)
    from paper_2111_13094_amd import sdmm
    wl = synth.workload("cells4k", scale=8 / 4096, seed=8)
    C = wl["grid"].n_cells
    b = synth.workload_batch(wl)
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    beta = 1e-3
    early = synth.copy_mix(mix)
    orc.fit(orc.Opts(K=16, iters=2, prior_mode=1, prior_scale=beta), b.offsets, b.samples, early,
            orc.new_state(C, 16))
    status = orc.fit(orc.Opts(K=16, iters=400, prior_mode=1, prior_scale=beta), b.offsets, b.samples, mix,
                     orc.new_state(C, 16))
    o = sdmm.default_opts(16, prior_mode=sdmm.PRIOR_FIXED, prior_scale=beta)
    off, smp = dev.from_numpy(b.offsets).cuda(), dev.from_numpy(b.samples).cuda()
    g_fix = {k: v.cpu().numpy() for k, v in sdmm.fit_grad(off, smp, to_torch(mix), o).items()}
    g_early = {k: v.cpu().numpy() for k, v in sdmm.fit_grad(off, smp, to_torch(early), o).items()}
    # a dead component keeps its mean and covariance, so F is not stationary in it
    live = [c for c in range(C) if not status[c] & orc.DEAD_COMPONENT]
    assert len(live) >= C // 2
    for key in ("alpha", "mu_pos", "L"):
        for c in live:
            ratio = np.abs(g_fix[key][c]).max() / np.abs(g_early[key][c]).max()
            assert ratio < 2e-3, (key, c, ratio)
