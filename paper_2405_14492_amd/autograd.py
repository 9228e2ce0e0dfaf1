"""torch.autograd.Function for the FSA negative log-likelihood.

forward: fsa_nll_grad without gradient (SLQ log-det + quadratic term from the
block PCG solves); backward: fsa_grad, the library's backward pass, which
reuses those solves and the preconditioned probes for the stochastic trace
estimate of eq. NEGLLDNEGLLFSA.  The parameter vector is
(sigma1^2, rho, sigma^2); optimise in log space by passing exp(phi).
"""
from __future__ import annotations

import torch

from . import fsa as F


class FSANLL(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, model: "F.FSA", cov: int):
        th = [float(v) for v in theta.detach().cpu().tolist()]
        nll, _, st = model.nll_grad(theta=(cov, *th), with_grad=False)
        ctx.model = model
        ctx.stats = st
        return theta.new_tensor(nll)

    @staticmethod
    def backward(ctx, g):
        grad, st = ctx.model.grad()
        ctx.stats.update({"grad_trace": st["grad_trace"], "grad_quad": st["grad_quad"]})
        return g * g.new_tensor(grad), None, None


def fsa_nll(theta: torch.Tensor, model: "F.FSA", cov: int) -> torch.Tensor:
    return FSANLL.apply(theta, model, cov)


def fit_lbfgs(model: "F.FSA", theta0, cov: int, steps: int = 20, lr: float = 1.0, history: int = 10):
    """Minimise the NLL over log(sigma1^2, rho, sigma^2) with torch L-BFGS.
    Returns (theta, trace of (nll, theta) per closure evaluation)."""
    phi = torch.tensor([float(v) for v in theta0], dtype=torch.float64).log().requires_grad_(True)
    opt = torch.optim.LBFGS([phi], lr=lr, max_iter=1, history_size=history, line_search_fn="strong_wolfe")
    trace = []

    def closure():
        opt.zero_grad()
        th = phi.exp()
        try:
            val = fsa_nll(th, model, cov)
            val.backward()
        except F.FsaError as e:
            # an infeasible trial point (e.g. breakdown at an extreme step):
            # report +inf so the line search backs off
            trace.append((float("inf"), th.detach().tolist(), str(e)))
            phi.grad = torch.zeros_like(phi)
            return phi.new_tensor(float("inf"))
        trace.append((float(val), th.detach().tolist()))
        return val.detach()

    for _ in range(steps):
        opt.step(closure)
    return phi.detach().exp().tolist(), trace
