"""Differentiable solve: ``torch.autograd.Function`` over the HIP library.

Forward: u = solve(dL_sigma u = f).  Backward (implicit-function theorem on
dL_sigma(u) = f, all faces Dirichlet, where dL is symmetric):
    lambda = solve(dL_sigma lambda = dLoss/du)   (adjoint solve, lambda = 0 on
                                                  Dirichlet nodes)
    dLoss/df     = lambda
    dLoss/dsigma = -C/(2h^2) sum_k w_k (u_k - u_m)(lambda_m - lambda_k)
Only the converged forward solution is kept for the backward pass; no
per-cycle state is stored.
"""
import torch

from . import sgml


class SGMLSolve(torch.autograd.Function):
    """u = SGMLSolve.apply(f, sigma, plan, G, opts).

    ``plan`` is an ``sgml.Plan`` on all-Dirichlet faces; ``sigma`` is the
    coefficient tensor bound to it (or None for sigma = 1); ``G`` the Dirichlet
    values or None; ``opts`` a dict of solve options (tol, max_cycles,
    precision, ...), used for the forward and the adjoint solves.
    """

    @staticmethod
    def forward(ctx, f, sigma, plan, G, opts):
        opts = dict(opts or {})
        if sigma is not plan.sigma:
            plan.set_coeffs(sigma)
        u, st = plan.solve(f.detach(), None if G is None else G.detach(), **opts)
        ctx.plan, ctx.opts, ctx.stats = plan, opts, st
        ctx.has_sigma = sigma is not None
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        (u,) = ctx.saved_tensors
        plan = ctx.plan
        lam, _ = plan.adjoint(grad_u.detach().contiguous(), **ctx.opts)
        grad_f = lam if ctx.needs_input_grad[0] else None
        grad_sigma = None
        if ctx.has_sigma and ctx.needs_input_grad[1]:
            grad_sigma = plan.coeff_grad(u, lam)
        return grad_f, grad_sigma, None, None, None


def solve(f, sigma, plan, G=None, **opts):
    """Differentiable solve with respect to f and sigma."""
    return SGMLSolve.apply(f, sigma, plan, G, opts)
