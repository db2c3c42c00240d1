"""GPU parity of the adjoint (sdmm_fit_grad through the C ABI) against the oracle's
objective and closed-form gradient, plus the stationarity check it is used for, for the
default pass (FP32 tangent coordinates and products, compensated sums, FP64 quadratic
form) and the FP64 verification mode. Tolerances are stated per test."""
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


TRI = [(d, e) for d in range(5) for e in range(d + 1)]


def _lower(v):
    M = np.zeros((5, 5))
    for i, (d, e) in enumerate(TRI):
        M[d, e] = v[i]
    return M


def _kappa(cov15):
    """Condition number of the component's correlation matrix."""
    S = _lower(cov15)
    S = S + np.tril(S, -1).T
    sd = np.sqrt(np.diag(S))
    return np.linalg.cond(S / np.outer(sd, sd))


def _whitened(g, cov, K):
    """Per component: L^T [g_delta; g_mu_pos] (the gradient with respect to the mean in
    units of the component's standard deviations) and L^T tril(g_L) (with respect to a
    relative change of L), with L the Cholesky factor of the component's covariance."""
    wm, wl = np.zeros((K, 5)), np.zeros((K, 5, 5))
    for k in range(K):
        S = _lower(cov[k])
        L = np.linalg.cholesky(S + np.tril(S, -1).T)
        wm[k] = L.T @ np.concatenate([g["delta"].reshape(K, 2)[k], g["mu_pos"].reshape(K, 3)[k]])
        wl[k] = L.T @ _lower(g["L"].reshape(K, 15)[k])
    return wm, wl


def _parity(dev, orc, flags):
    from paper_2111_13094_amd import sdmm
    wl, b, mix = _problem(orc)
    C, K = wl["grid"].n_cells, 16
    beta = 0.02
    o = sdmm.default_opts(K, prior_mode=sdmm.PRIOR_FIXED, prior_scale=beta, flags=flags)
    out = sdmm.fit_grad(dev.from_numpy(b.offsets).cuda(), dev.from_numpy(b.samples).cuda(), to_torch(mix), o)
    dev.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    assert (got["status"] == 0).all()
    oo = orc.Opts(K=K, prior_mode=1, prior_scale=beta)
    cov = mix["cov"].reshape(C, K, 15)
    for c in range(C):
        i0, i1 = b.offsets[c], b.offsets[c + 1]
        F = orc.objective(oo, b.samples, i0, i1, mix, beta, cell=c)
        g = orc.grad(oo, b.samples, i0, i1, mix, beta, cell=c)
        gg = {key: got[key][c] for key in ("alpha", "mu_pos", "delta", "L")}
        yield c, cov[c], got["F"][c], F, gg, g


def test_gradient_parity(dev, orc):
    """FP32 pass (FP64 quadratic form): F within 1e-6 relative; the weight-logit block
    within 1e-4 of its largest entry; the mean and factor blocks compared whitened
    (see _whitened) within 2e-4, on components whose correlation matrix has condition
    number <= 1e5. Beyond that the FP32 tangent coordinates and products (relative
    rounding 2^-24) are amplified by about the condition number in Sigma^-1, and those
    components are checked by the FP64 mode below."""
    print("case: adjoint on 27 cells, FP32 pass", flush=True)
    worst = {"F": 0.0, "alpha": 0.0, "mean": 0.0, "L": 0.0}
    n_checked = n_all = 0
    for c, cov, Fg, F, gg, g in _parity(dev, orc, 0):
        K = cov.shape[0]
        worst["F"] = max(worst["F"], abs(Fg - F) / abs(F))
        worst["alpha"] = max(worst["alpha"], np.abs(gg["alpha"] - g["alpha"]).max() / np.abs(g["alpha"]).max())
        ok = np.array([_kappa(cov[k]) <= 1e5 for k in range(K)])
        n_checked += ok.sum()
        n_all += K
        wm_g, wl_g = _whitened(gg, cov, K)
        wm_o, wl_o = _whitened(g, cov, K)
        worst["mean"] = max(worst["mean"], np.abs(wm_g - wm_o)[ok].max() / np.abs(wm_o[ok]).max())
        worst["L"] = max(worst["L"], np.abs(wl_g - wl_o)[ok].max() / np.abs(wl_o[ok]).max())
    print(worst, f"{n_checked} of {n_all} components well conditioned")
    assert worst["F"] <= 1e-6 and worst["alpha"] < 1e-4, worst
    assert worst["mean"] < 2e-4 and worst["L"] < 2e-4, worst
    assert n_checked >= 0.9 * n_all


def test_gradient_parity_fp64_mode(dev, orc):
    """FP64 verification mode: every block of every component within 1e-7 of the block's
    largest entry (FP64 rounding, 2^-53, amplified by the condition number of the worst
    component, ~3e7 here), F within 1e-10 relative."""
    print("case: adjoint on 27 cells, FP64 pass", flush=True)
    from paper_2111_13094_amd import sdmm
    worst = {"F": 0.0, "alpha": 0.0, "mu_pos": 0.0, "delta": 0.0, "L": 0.0}
    for c, cov, Fg, F, gg, g in _parity(dev, orc, sdmm.FLAG_FP64_SUMS):
        worst["F"] = max(worst["F"], abs(Fg - F) / abs(F))
        for key in ("alpha", "mu_pos", "delta", "L"):
            ref = g[key].reshape(gg[key].shape)
            worst[key] = max(worst[key], np.abs(gg[key] - ref).max() / np.abs(ref).max())
    print(worst)
    assert worst["F"] <= 1e-10, worst
    for key in ("alpha", "mu_pos", "delta", "L"):
        assert worst[key] < 1e-7, (key, worst)


def _fixed_point(orc):
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
    return C, b, mix, early, status, beta


def test_gradient_vanishes_at_a_batch_em_fixed_point_fp32(dev, orc):
    """At a fixed point of batch MAP-EM (mean offsets m = 0, so the transfer Jacobian is
    the identity) the updates of the weights, positional means and covariances are exact
    maximisers of F, so those gradient blocks vanish; they are compared with the same
    blocks two EM steps in (per component, against the cell's largest early entry). The
    FP32 pass resolves this on components whose correlation matrix has condition number
    <= 1e3 (ratio < 2e-3); with parallax data many converged components are far more
    correlated than that, and the FP64 mode covers them."""
    print("case: stationarity after 400 EM iterations (8 cells), FP32 pass", flush=True)
    from paper_2111_13094_amd import sdmm
    C, b, mix, early, status, beta = _fixed_point(orc)
    o = sdmm.default_opts(16, prior_mode=sdmm.PRIOR_FIXED, prior_scale=beta)
    off, smp = dev.from_numpy(b.offsets).cuda(), dev.from_numpy(b.samples).cuda()
    g_fix = {k: v.cpu().numpy() for k, v in sdmm.fit_grad(off, smp, to_torch(mix), o).items()}
    g_early = {k: v.cpu().numpy() for k, v in sdmm.fit_grad(off, smp, to_torch(early), o).items()}
    # a dead component keeps its mean and covariance, so F is not stationary in it
    live = [c for c in range(C) if not status[c] & orc.DEAD_COMPONENT]
    assert len(live) >= C // 2
    cov = mix["cov"].reshape(C, 16, 15)
    worst, n_checked = {}, 0
    for key in ("alpha", "mu_pos", "L"):
        r = 0.0
        for c in live:
            for k in range(16):
                if _kappa(cov[c, k]) > 1e3:
                    continue
                n_checked += key == "alpha"
                r = max(r, np.abs(g_fix[key][c][k]).max() / np.abs(g_early[key][c]).max())
        worst[key] = r
    print("fixed point / early gradient, worst:", worst, f"over {n_checked} components")
    for key, ratio in worst.items():
        assert ratio < 2e-3, (key, ratio)
    assert n_checked >= len(live) * 2


def test_gradient_vanishes_at_a_batch_em_fixed_point_fp64(dev, orc):
    """FP64 mode at the same fixed point, on the components of the live cells whose
    correlation matrix has condition number kappa <= 1e5: the oracle's gradient there is
    below 1e-4 of the early one (the fit has converged to that level: the weights
    converge slowest), and the device gradient equals the oracle's within 1e-7 of the
    early gradient, so the device adjoint resolves stationarity wherever the oracle does.
    Beyond kappa ~ 1e5 the covariance gradient Sigma^-1 (...) Sigma^-1 cancels with
    FP64 rounding amplified by kappa^2 in both implementations."""
    print("case: stationarity after 400 EM iterations (8 cells), FP64 pass", flush=True)
    from paper_2111_13094_amd import sdmm
    from paper_2111_13094_amd import autograd
    C, b, mix, early, status, beta = _fixed_point(orc)
    o = sdmm.default_opts(16, prior_mode=sdmm.PRIOR_FIXED, prior_scale=beta)
    off, smp = dev.from_numpy(b.offsets).cuda(), dev.from_numpy(b.samples).cuda()
    # the stationarity check of the autograd module takes the FP64 pass
    g_fix = {k: v.cpu().numpy() for k, v in autograd.stationarity(to_torch(mix), off, smp, o).items()}
    g_early = {k: v.cpu().numpy() for k, v in autograd.stationarity(to_torch(early), off, smp, o).items()}
    live = [c for c in range(C) if not status[c] & orc.DEAD_COMPONENT]
    assert len(live) >= C // 2
    oo = orc.Opts(K=16, prior_mode=1, prior_scale=beta)
    cov = mix["cov"].reshape(C, 16, 15)
    worst_orc, worst_diff, n_checked = {}, {}, 0
    for key in ("alpha", "mu_pos", "L"):
        ro = rd = 0.0
        for c in live:
            i0, i1 = b.offsets[c], b.offsets[c + 1]
            ref = orc.grad(oo, b.samples, i0, i1, mix, beta, cell=c)[key].reshape(g_fix[key][c].shape)
            scale = np.abs(g_early[key][c]).max()
            for k in range(16):
                if _kappa(cov[c, k]) > 1e5:
                    continue
                n_checked += key == "alpha"
                ro = max(ro, np.abs(ref[k]).max() / scale)
                rd = max(rd, np.abs(g_fix[key][c][k] - ref[k]).max() / scale)
        worst_orc[key], worst_diff[key] = ro, rd
    print("oracle fixed point / early:", worst_orc, "device - oracle at the fixed point / early:", worst_diff,
          f"over {n_checked} components")
    assert n_checked >= len(live) * 8
    for key in worst_orc:
        assert worst_orc[key] < 1e-4, (key, worst_orc)
        assert worst_diff[key] < 1e-7, (key, worst_diff)


def _fd_params(rng, K, n_per_comp=1):
    """(block, component, index) triples to difference: for four random components of a
    cell, one weight logit, one positional coordinate, one tangent direction and two
    entries of L."""
    out = []
    for k in rng.choice(K, 4, replace=False):
        out += [("alpha", k, 0), ("mu_pos", k, int(rng.integers(3))), ("delta", k, int(rng.integers(2)))]
        out += [("L", k, int(t)) for t in rng.choice(15, 2, replace=False)]
    return out


def _objective_at(orc, oo, smp, i0, i1, mix, beta, c, K, block, k, idx, h):
    """F of cell c with one parameter moved by h, in the parameterisation of the
    adjoint (logits, positions, tangent perturbation of mu_dir, Cholesky factor)."""
    m = {key: np.ascontiguousarray(v.reshape(-1, K * (v.size // (mix["pi"].size)))[c]).ravel().copy()
         for key, v in mix.items()}
    if block == "alpha":
        a = np.log(m["pi"])
        a[k] += h
        e = np.exp(a - a.max())
        m["pi"] = e / e.sum()
    elif block == "mu_pos":
        m["mu_pos"][3 * k + idx] += h
    elif block == "delta":
        dl = np.zeros(2)
        dl[idx] = h
        w = orc.exp_map(m["mu_dir"][3 * k:3 * k + 3].copy(), dl)
        m["mu_dir"][3 * k:3 * k + 3] = w / np.linalg.norm(w)
    else:
        L = np.linalg.cholesky(_lower(m["cov"][15 * k:15 * k + 15]) + np.tril(_lower(m["cov"][15 * k:15 * k + 15]), -1).T)
        Lp = np.array([L[d, e] for (d, e) in TRI])
        Lp[idx] += h
        U = _lower(Lp)
        S = U @ U.T
        m["cov"][15 * k:15 * k + 15] = [S[d, e] for (d, e) in TRI]
    return orc.objective(oo, smp, i0, i1, m, beta)


def test_adjoint_at_the_4096_cell_state_after_8_batches(dev, orc):
    """The adjoint's own workload: the 4096-cell state after 8 batches (eta = 0.1), the
    gradient of F on the 9th batch for every cell, fixed prior strength 1e-3 (the
    benchmark's configuration). On cells 0-63 against the oracle's closed form
    (Sec. 4.3 objective): the FP64 pass on every component within 1e-7 of each block's
    largest entry, the FP32 pass within 2e-4 (whitened) where the component's correlation
    matrix has condition number <= 1e5; and both the oracle's and the FP64 pass's
    gradients against FP64 central differences of the oracle's F (20 parameters per
    cell, relative step 1e-6) within 1e-6 of the block's largest entry."""
    print("case: adjoint at the 4096-cell state after 8 batches, 64 cells vs oracle and FD", flush=True)
    from paper_2111_13094_amd import sdmm
    wl = synth.workload("cells4k")
    C, K = wl["grid"].n_cells, 16
    mix = to_torch(synth.initial_mixtures(wl["box_lo"], wl["box_size"], K))
    st = sdmm.new_state(C, K)
    for j in range(8):
        b = synth.workload_batch(wl, j)
        sdmm.fit_mixtures(dev.from_numpy(b.offsets).cuda(), dev.from_numpy(b.samples).cuda(), mix, st,
                          sdmm.default_opts(K, eta=0.1))
    b = synth.workload_batch(wl, 8)
    off, smp = dev.from_numpy(b.offsets).cuda(), dev.from_numpy(b.samples).cuda()
    beta = 1e-3
    g32 = {k: v.cpu().numpy() for k, v in sdmm.fit_grad(
        off, smp, mix, sdmm.default_opts(K, prior_mode=sdmm.PRIOR_FIXED, prior_scale=beta)).items()}
    g64 = {k: v.cpu().numpy() for k, v in sdmm.fit_grad(
        off, smp, mix, sdmm.default_opts(K, prior_mode=sdmm.PRIOR_FIXED, prior_scale=beta,
                                         flags=sdmm.FLAG_FP64_SUMS)).items()}
    dev.cuda.synchronize()
    host = {k: v.cpu().numpy() for k, v in mix.items()}
    oo = orc.Opts(K=K, prior_mode=1, prior_scale=beta)
    cov = host["cov"].reshape(C, K, 15)
    rng = np.random.default_rng(5)
    worst = {"F32": 0.0, "F64": 0.0, "alpha32": 0.0, "mean32": 0.0, "L32": 0.0, "g64": 0.0, "fd_orc": 0.0,
             "fd_gpu": 0.0}
    n_ok = n_all = 0
    h = 1e-6
    for c in range(64):
        assert g32["status"][c] == 0 and g64["status"][c] == 0, c
        i0, i1 = b.offsets[c], b.offsets[c + 1]
        F = orc.objective(oo, b.samples, i0, i1, host, beta, cell=c)
        g = orc.grad(oo, b.samples, i0, i1, host, beta, cell=c)
        worst["F32"] = max(worst["F32"], abs(g32["F"][c] - F) / abs(F))
        worst["F64"] = max(worst["F64"], abs(g64["F"][c] - F) / abs(F))
        for key in ("alpha", "mu_pos", "delta", "L"):
            ref = g[key].reshape(g64[key][c].shape)
            worst["g64"] = max(worst["g64"], np.abs(g64[key][c] - ref).max() / np.abs(ref).max())
        worst["alpha32"] = max(worst["alpha32"], np.abs(g32["alpha"][c] - g["alpha"]).max() / np.abs(g["alpha"]).max())
        ok = np.array([_kappa(cov[c, k]) <= 1e5 for k in range(K)])
        n_ok += ok.sum()
        n_all += K
        gg = {key: g32[key][c] for key in ("alpha", "mu_pos", "delta", "L")}
        wm_g, wl_g = _whitened(gg, cov[c], K)
        wm_o, wl_o = _whitened(g, cov[c], K)
        if ok.any():
            worst["mean32"] = max(worst["mean32"], np.abs(wm_g - wm_o)[ok].max() / np.abs(wm_o[ok]).max())
            worst["L32"] = max(worst["L32"], np.abs(wl_g - wl_o)[ok].max() / np.abs(wl_o[ok]).max())
        # central differences of the oracle's F
        for block, k, idx in _fd_params(rng, K):
            fp = _objective_at(orc, oo, b.samples, i0, i1, host, beta, c, K, block, k, idx, h)
            fm = _objective_at(orc, oo, b.samples, i0, i1, host, beta, c, K, block, k, idx, -h)
            fd = (fp - fm) / (2 * h)
            ref = g[block].reshape(g64[block][c].shape)
            scale = np.abs(ref).max()
            worst["fd_orc"] = max(worst["fd_orc"], abs(fd - ref[k].ravel()[idx]) / scale)
            worst["fd_gpu"] = max(worst["fd_gpu"], abs(fd - g64[block][c][k].ravel()[idx]) / scale)
    print({k: "%.2e" % v for k, v in worst.items()}, f"{n_ok} of {n_all} components with kappa <= 1e5")
    assert worst["F32"] <= 1e-6 and worst["F64"] <= 1e-10, worst
    assert worst["g64"] < 1e-7 and worst["alpha32"] < 1e-4, worst
    assert worst["mean32"] < 2e-4 and worst["L32"] < 2e-4, worst
    assert worst["fd_orc"] < 1e-6 and worst["fd_gpu"] < 1e-6, worst
