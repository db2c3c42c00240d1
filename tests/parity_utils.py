"""Helpers for GPU-vs-oracle parity tests: moving mixtures between numpy and torch,
and frame-invariant comparisons of fitted parameters.

Tolerances (per E+M step from identical FP64 parameters, FP32 E-step vs FP64 oracle):
directional mean angle <= 1e-5 rad; weights and positional means relative <= 1e-4 (with
an absolute floor); covariances relative <= 1e-4 in the Frobenius norm (the stated bar,
"cov_fro") and, stricter, <= 1e-4 in the oracle covariance's own metric
(|| L^-1 (S_gpu - S_orc) L^-T ||_2 with S_orc = L L^T, "cov"). The second measure divides
by the smallest eigenvalue of the oracle covariance; for cells with fewer than 64
positive weights that eigenvalue is set by the prior, and FP32 rounding of the data
scatter shows in it at up to SMALL_CELL_METRIC (a documented reading with its
derivation). Trajectories over many iterations or batches <= 1e-3 (EM amplifies FP32
rounding)."""
from __future__ import annotations

import numpy as np

TRI = [(d, e) for d in range(5) for e in range(d + 1)]


def unpack(c):
    S = np.zeros((5, 5))
    for i, (d, e) in enumerate(TRI):
        S[d, e] = S[e, d] = c[i]
    return S


def pack(S):
    return np.array([S[d, e] for (d, e) in TRI])


def to_torch(mix: dict, device="cuda"):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(device) for k, v in mix.items()}


def to_numpy(mix: dict):
    return {k: v.detach().cpu().numpy().copy() for k, v in mix.items()}


def state_to_torch(st: dict, device="cuda"):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(device) for k, v in st.items()}


def frame(mu):
    """Same construction the library documents for R_mu (Duff et al. 2017), used only to
    express both sides' tangent covariances in a common frame."""
    sg = 1.0 if np.copysign(1.0, mu[2]) > 0 else -1.0
    a = -1.0 / (sg + mu[2])
    b = mu[0] * mu[1] * a
    t1 = np.array([1.0 + sg * mu[0] * mu[0] * a, sg * b, -sg * mu[0]])
    t2 = np.array([b, sg + mu[1] * mu[1] * a, -mu[1]])
    return np.stack([t1, t2, mu])


def to_frame(S, mu_from, mu_to):
    """Express a 5x5 tangent covariance stored in the frame of mu_from in the frame of
    mu_to (both means within rounding of each other)."""
    Rf, Rt = frame(mu_from), frame(mu_to)
    G = Rt[:2] @ Rf[:2].T
    T = np.eye(5)
    T[:2, :2] = G
    return T @ S @ T.T


def metric_error(S_test, S_ref):
    L = np.linalg.cholesky(S_ref)
    Li = np.linalg.inv(L)
    return np.linalg.norm(Li @ (S_test - S_ref) @ Li.T, 2)


SMALL_CELL_METRIC = 2e-3   # whitened covariance metric for cells with M < 64
SMALL_CELL_M = 64


def positive_counts(samples, offsets):
    """M = #{w > 0} per cell."""
    return np.array([(samples[6, offsets[c]:offsets[c + 1]] > 0).sum() for c in range(offsets.size - 1)])


def compare_mixtures(got: dict, ref: dict, K: int, cells=None, rtol=1e-4, ang_tol=1e-5, pi_abs=1e-7):
    """Returns a dict of the worst errors over the given cells (all by default)."""
    C = ref["pi"].size // K
    cells = range(C) if cells is None else cells
    worst = {"pi": 0.0, "mu_dir": 0.0, "mu_pos": 0.0, "cov": 0.0, "cov_fro": 0.0}
    for c in cells:
        for k in range(K):
            g = c * K + k
            pr, pg = ref["pi"][g], got["pi"][g]
            worst["pi"] = max(worst["pi"], abs(pg - pr) / (rtol * abs(pr) + pi_abs) * rtol)
            mr, mg = ref["mu_dir"][3 * g:3 * g + 3], got["mu_dir"][3 * g:3 * g + 3]
            worst["mu_dir"] = max(worst["mu_dir"], np.arctan2(np.linalg.norm(np.cross(mr, mg)), mr @ mg))
            xr, xg = ref["mu_pos"][3 * g:3 * g + 3], got["mu_pos"][3 * g:3 * g + 3]
            worst["mu_pos"] = max(worst["mu_pos"], np.abs(xg - xr).max() / max(np.abs(xr).max(), 1e-3))
            Sr = unpack(ref["cov"][15 * g:15 * g + 15])
            Sg = to_frame(unpack(got["cov"][15 * g:15 * g + 15]), mg, mr)
            worst["cov"] = max(worst["cov"], metric_error(Sg, Sr))
            worst["cov_fro"] = max(worst["cov_fro"], np.linalg.norm(Sg - Sr) / np.linalg.norm(Sr))
    return worst


def assert_close(worst: dict, rtol=1e-4, ang_tol=1e-5, what="", metric_tol=None):
    """rtol bounds pi, mu_pos and cov_fro; metric_tol (default rtol) the whitened
    covariance metric; ang_tol the directional mean angle in radians."""
    metric_tol = rtol if metric_tol is None else metric_tol
    tol = {"mu_dir": ang_tol, "cov": metric_tol}
    bad = {k: v for k, v in worst.items() if v > tol.get(k, rtol)}
    assert not bad, f"{what} parity failed: {worst}"


def assert_cells_close(got: dict, ref: dict, K: int, cells, m_pos, what="", rtol=1e-4, ang_tol=1e-5):
    """Per-cell parity at the stated bar; cells with fewer than SMALL_CELL_M positive
    weights take SMALL_CELL_METRIC for the whitened covariance metric only."""
    for c in cells:
        worst = compare_mixtures(got, ref, K, cells=[c])
        small = m_pos[c] < SMALL_CELL_M
        print(c, int(m_pos[c]), {k: "%.2e" % v for k, v in worst.items()})
        assert_close(worst, rtol=rtol, ang_tol=ang_tol, metric_tol=SMALL_CELL_METRIC if small else rtol,
                     what=f"{what} cell {c} (M={m_pos[c]})")


def draw_radius(m, Sc, u):
    """|nu| of a draw nu = m + chol(Sc) z, z by Box-Muller from the draw's uniforms u[1]
    (mapped to (0, 1] as 1 - u[1]) and u[2]: the quantity the cut-locus discard tests
    (Sec. 3.1, draws with |nu| >= pi are discarded). Sc is the packed 2x2 covariance."""
    L = np.linalg.cholesky(np.array([[Sc[0], Sc[1]], [Sc[1], Sc[2]]]))
    rad = np.sqrt(-2.0 * np.log(1.0 - u[1]))
    z = rad * np.array([np.cos(2.0 * np.pi * u[2]), np.sin(2.0 * np.pi * u[2])])
    return float(np.linalg.norm(np.asarray(m, dtype=np.float64) + L @ z))


# a draw whose validity differs between the FP32 device and the FP64 oracle must lie
# this close to the cut locus |nu| = pi
CUT_LOCUS_BAND = 1e-5
