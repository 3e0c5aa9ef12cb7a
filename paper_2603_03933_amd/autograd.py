"""torch.autograd interface to the Landau-Brazovskii energy of eq. lb_energy.

`energy(plan, psi, tau, gamma)` returns E for each of the plan's `batch`
fields and is differentiable in psi, tau and gamma up to second order. Torch
sees E as a function of the N grid values of each field, with the sum over
every k including k = 0 (on zero-mean fields it is the paper's E):

  dE/dpsi_x        = (F_N^{-1} Lambda psi_hat + F'(psi))_x / N   (lb_energy_grad_raw)
  d2E/dpsi^2 . v   = (F_N^{-1} Lambda F_N v + Gamma'(psi) v) / N  (lb_hessvec_raw)
  dE/dtau, dE/dgamma and d<G, dE/dpsi>/d(tau, gamma)            (lb_param_grad)
  d(a dE/dtau + b dE/dgamma)/dpsi                                (lb_param_grad_vjp)

Every derivative is computed by the library; the only torch arithmetic here
is the chain rule: products of those derivatives with incoming gradients.
The paper's convention (projected gradient in Psi_hat coordinates, norms in
RMS) is the library's lb_energy_grad; the two differ by the mean and a factor N.
"""
from __future__ import annotations

import torch

from . import lb


def _params(tau: torch.Tensor, gamma: torch.Tensor, xi: float, q: float, batch: int):
    t = tau.detach().reshape(-1).tolist()
    g = gamma.detach().reshape(-1).tolist()
    if len(t) == 1:
        t = t * batch
    if len(g) == 1:
        g = g * batch
    if len(t) != batch or len(g) != batch:
        raise ValueError(f"tau and gamma need 1 or {batch} entries")
    return [lb.Params(a, b, xi, q) for a, b in zip(t, g)]


def _expand(x: torch.Tensor, like: torch.Tensor):
    """Per-instance values [B] broadcast over fields of shape [B, ...]."""
    return x.reshape(x.shape[0], *([1] * (like.dim() - 1)))


def _reduce_like(g: torch.Tensor, param: torch.Tensor):
    """Per-instance gradient [B] summed to the shape of a broadcast parameter."""
    return g.sum().reshape(param.shape) if param.numel() == 1 else g.reshape(param.shape)


class _ParamGrad(torch.autograd.Function):
    """(dE/dtau, dE/dgamma) per instance; its psi-gradient comes from lb_param_grad_vjp."""

    @staticmethod
    def forward(ctx, psi, plan):
        ctx.save_for_backward(psi)
        ctx.plan = plan
        return plan.lb_param_grad(psi).reshape(plan.batch, 4)[:, :2].contiguous()

    @staticmethod
    def backward(ctx, g2):
        (psi,) = ctx.saved_tensors
        return ctx.plan.lb_param_grad_vjp(psi, g2.contiguous().reshape(-1)), None


class _GradRaw(torch.autograd.Function):
    """dE/dpsi (raw grid coordinates); its backward is the Hessian product."""

    @staticmethod
    def forward(ctx, psi, tau, gamma, plan, xi, q):
        ctx.save_for_backward(psi, tau, gamma)
        ctx.plan, ctx.xi, ctx.q = plan, xi, q
        _, g = plan.lb_energy_grad_raw(_params(tau, gamma, xi, q, plan.batch), psi)
        return g

    @staticmethod
    def backward(ctx, G):
        psi, tau, gamma = ctx.saved_tensors
        plan = ctx.plan
        G = G.contiguous()
        dpsi = plan.lb_hessvec_raw(_params(tau, gamma, ctx.xi, ctx.q, plan.batch), psi, G)
        m = plan.lb_param_grad(psi, G).reshape(plan.batch, 4)
        dtau = _reduce_like(m[:, 2], tau).to(tau.dtype)
        dgamma = _reduce_like(m[:, 3], gamma).to(gamma.dtype)
        return dpsi, dtau.to(tau.device), dgamma.to(gamma.device), None, None, None


class _Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi, tau, gamma, plan, xi, q):
        ctx.save_for_backward(psi, tau, gamma)
        ctx.plan, ctx.xi, ctx.q = plan, xi, q
        E, _ = plan.lb_energy_grad(_params(tau, gamma, xi, q, plan.batch), psi, want_grad=False)
        return E

    @staticmethod
    def backward(ctx, gE):
        psi, tau, gamma = ctx.saved_tensors
        plan = ctx.plan
        dpsi = dtau = dgamma = None
        if ctx.needs_input_grad[0]:
            dpsi = _expand(gE, psi) * _GradRaw.apply(psi, tau, gamma, plan, ctx.xi, ctx.q)
        if ctx.needs_input_grad[1] or ctx.needs_input_grad[2]:
            mg = _ParamGrad.apply(psi, plan)
            dtau = _reduce_like(gE * mg[:, 0].to(gE.device), tau).to(tau.device)
            dgamma = _reduce_like(gE * mg[:, 1].to(gE.device), gamma).to(gamma.device)
        return dpsi, dtau, dgamma, None, None, None


def energy(plan: "lb.Plan", psi: torch.Tensor, tau, gamma, xi: float = 1.0, q: float = 1.0) -> torch.Tensor:
    """E of each field: psi is [plan.batch, *grid] float64 on the GPU (or [*grid]
    for a plan of batch 1); tau and gamma are floats or tensors with 1 or
    plan.batch entries. Returns a [plan.batch] tensor."""
    if psi.dim() == len(plan.n):
        psi = psi.unsqueeze(0)
    if tuple(psi.shape) != (plan.batch, *plan.n):
        raise ValueError(f"psi has shape {tuple(psi.shape)}, plan expects {(plan.batch, *plan.n)}")
    tau = torch.as_tensor(tau, dtype=torch.float64)
    gamma = torch.as_tensor(gamma, dtype=torch.float64)
    return _Energy.apply(psi.contiguous(), tau, gamma, plan, float(xi), float(q))
