"""Helpers for GPU-vs-oracle parity tests: moving mixtures between numpy and torch,
and frame-invariant comparisons of fitted parameters.

Tolerances (per E+M step from identical FP64 parameters, FP32 E-step vs FP64 oracle):
directional mean angle <= 1e-5 rad; weights and positional means relative <= 1e-4 (with
an absolute floor); covariances <= 1e-4 in the oracle covariance's own metric
(|| L^-1 (S_gpu - S_orc) L^-T ||_2 with S_orc = L L^T); trajectories over many
iterations or batches <= 1e-3 (EM amplifies FP32 rounding)."""
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


def compare_mixtures(got: dict, ref: dict, K: int, cells=None, rtol=1e-4, ang_tol=1e-5, pi_abs=1e-7):
    """Returns a dict of the worst errors over the given cells (all by default)."""
    C = ref["pi"].size // K
    cells = range(C) if cells is None else cells
    worst = {"pi": 0.0, "mu_dir": 0.0, "mu_pos": 0.0, "cov": 0.0}
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
    return worst


def assert_close(worst: dict, rtol=1e-4, ang_tol=1e-5, what=""):
    bad = {k: v for k, v in worst.items() if (v > ang_tol if k == "mu_dir" else v > rtol)}
    assert not bad, f"{what} parity failed: {worst}"
