"""torch.autograd binding of the adjoint: the weighted penalised log-likelihood of the
fitted mixtures as a differentiable function of unconstrained parameters.

Per cell c, with pi = softmax(alpha), mu_dir = exp_{mu0}(delta) (the exp map of Sec. 3.1
of Dodik et al. in the frame of mu0), mu_pos, and Sigma = L L^T,

    F_c = sum_i (w_i / W) log sum_k pi_k N5(y_ik; 0, Sigma_k)
          + sum_k [beta q log pi_k - (beta a / 2) log det Sigma_k - (beta / 2) tr(B Sigma_k^-1)],

the objective whose maximiser is the MAP update of Sec. 4.3. The forward pass runs
sdmm_mixture_from_params, sdmm_fit_grad (value and gradient in one pass over the
samples) and sdmm_grad_to_params; the backward pass only scales the stored gradients by
the incoming per-cell gradient.
"""
from __future__ import annotations

import torch

from . import sdmm


class PenalisedLogLikelihood(torch.autograd.Function):
    """F per cell (float64 [C]) and the cell status (int32 [C], not differentiable) from
    alpha [C,K], delta [C,K,2], mu_pos [C,K,3], L [C,K,15] (float64, device); mu_dir0
    [C,K,3], the cell offsets, the samples and the options are constants."""

    @staticmethod
    def forward(ctx, alpha, delta, mu_pos, L, mu_dir0, cell_offsets, samples, opts, workspace=None):
        alpha, delta, mu_pos, L = (t.detach().contiguous() for t in (alpha, delta, mu_pos, L))
        mix, jac = sdmm.mixture_from_params(alpha, mu_dir0.contiguous(), delta, mu_pos, L)
        out = sdmm.fit_grad(cell_offsets, samples, mix, opts, workspace=workspace)
        sdmm.grad_to_params(L, jac, out["delta"], out["L"])
        ctx.save_for_backward(out["alpha"], out["delta"], out["mu_pos"], out["L"])
        ctx.mark_non_differentiable(out["status"])
        return out["F"], out["status"]

    @staticmethod
    def backward(ctx, grad_F, grad_status):
        g_alpha, g_delta, g_mu_pos, g_L = ctx.saved_tensors
        s = grad_F.to(torch.float64).reshape(-1, 1)
        return (g_alpha * s, g_delta * s.unsqueeze(-1), g_mu_pos * s.unsqueeze(-1), g_L * s.unsqueeze(-1),
                None, None, None, None, None)


def penalised_log_likelihood(params: dict, cell_offsets, samples, opts, workspace=None):
    """F per cell and the cell status for a parameter dict with keys alpha, delta, mu_pos,
    L, mu_dir0 (see PenalisedLogLikelihood)."""
    return PenalisedLogLikelihood.apply(params["alpha"], params["delta"], params["mu_pos"], params["L"],
                                        params["mu_dir0"], cell_offsets, samples, opts, workspace)


def params_from_mixture(mix: dict, n_cells: int, K: int, requires_grad=True) -> dict:
    """Refinement parameters at a mixture: alpha = log pi, L = chol(Sigma) (device
    kernel), delta = 0 about mu_dir0 = the mixture's directional means."""
    alpha, L, status = sdmm.params_from_mixture(mix, n_cells, K)
    if int((status != 0).sum()) != 0:
        raise ValueError("mixture has cells with unusable parameters (non-SPD covariance or weight <= 0)")
    p = {"alpha": alpha, "L": L,
         "delta": torch.zeros(n_cells, K, 2, dtype=torch.float64, device=alpha.device),
         "mu_pos": mix["mu_pos"].detach().reshape(n_cells, K, 3).clone(),
         "mu_dir0": mix["mu_dir"].detach().reshape(n_cells, K, 3).clone()}
    for k in ("alpha", "L", "delta", "mu_pos"):
        p[k].requires_grad_(requires_grad)
    return p


def mixture_from_params(params: dict) -> dict:
    """The mixture (flat float64 device arrays, as sdmm_fit_mixtures takes them) of a
    parameter dict."""
    with torch.no_grad():
        mix, _ = sdmm.mixture_from_params(params["alpha"].detach().contiguous(), params["mu_dir0"].contiguous(),
                                          params["delta"].detach().contiguous(),
                                          params["mu_pos"].detach().contiguous(), params["L"].detach().contiguous(),
                                          with_jac=False)
    return mix


def stationarity(mix: dict, cell_offsets, samples, opts, workspace=None) -> dict:
    """Gradient of F at fitted mixtures for checking EM stationarity (its blocks vanish at a
    fixed point of batch MAP-EM), from the FP64 pass (SDMM_FLAG_FP64_SUMS). The default FP32
    pass agrees with the closed-form gradient only on components whose correlation matrix
    has condition number <= 1e5, and resolves a fixed point only where it is <= 1e3: its
    FP32 tangent coordinates carry relative rounding 2^-24, which Sigma^-1 amplifies by
    about the condition number. Converged components with strong direction-position
    correlation exceed that, so the check always takes the FP64 pass. Returns the dict of
    sdmm.fit_grad."""
    o = type(opts).from_buffer_copy(opts)
    o.flags |= sdmm.FLAG_FP64_SUMS
    return sdmm.fit_grad(cell_offsets, samples, mix, o, workspace=workspace)


def refine(mix: dict, n_cells: int, K: int, cell_offsets, samples, opts, steps=10, lr=1e-3):
    """Gradient refinement of fitted mixtures: `steps` Adam ascent steps on
    (alpha, delta, mu_pos, L) of the summed F. Returns (refined mixture, F per cell
    before, F per cell after the last step, status)."""
    p = params_from_mixture(mix, n_cells, K)
    opt = torch.optim.Adam([p["alpha"], p["delta"], p["mu_pos"], p["L"]], lr=lr, maximize=True)
    N = samples.shape[1]
    ws = torch.empty(sdmm.workspace_bytes(n_cells, K, N, opts), dtype=torch.uint8, device=samples.device)
    F0 = None
    for _ in range(steps):
        opt.zero_grad()
        F, status = penalised_log_likelihood(p, cell_offsets, samples, opts, ws)
        if F0 is None:
            F0 = F.detach().clone()
        F.sum().backward()
        opt.step()
    with torch.no_grad():
        F1, status = penalised_log_likelihood(p, cell_offsets, samples, opts, ws)
    return mixture_from_params(p), F0, F1, status
