"""Differentiable solve: ``torch.autograd.Function`` over the HIP library.

Forward: u = solve(dL_sigma u = f).  Backward (implicit-function theorem on
dL_sigma(u) = f):
    lambda = solve(dL_sigma^T lambda = dLoss/du)   (adjoint solve, lambda = 0 on
                                                   Dirichlet nodes)
    dLoss/df     = lambda
    dLoss/dsigma = -sum_x lambda_x d(dL_sigma u)_x / dsigma
The adjoint and the coefficient gradient are the library's (sgml_adjoint,
sgml_coeff_grad).  Only the converged forward solution (and the
coefficient it was computed with) is kept for the backward pass; no
per-cycle state is stored.
"""
import torch

from . import sgml


def _bind(plan, sigma):
    """Bind `sigma` (or sigma = 1 for None) to the plan and rebuild its
    restricted coefficients.  Always rebuilt: the same tensor may have been
    changed in place since it was last bound."""
    plan.set_coeffs(None if sigma is None else sigma.detach())


class SGMLSolve(torch.autograd.Function):
    """u = SGMLSolve.apply(f, sigma, plan, G, opts).

    ``plan`` is an ``sgml.Plan``; ``sigma`` the coefficient tensor (or None
    for sigma = 1), bound to the plan for the forward solve and bound again
    for the backward solves, so several solves with different coefficients
    may share one plan before ``backward``; ``G`` the Dirichlet values or
    None; ``opts`` a dict of solve options (tol, max_cycles, precision, ...),
    used for the forward and the adjoint solves.  Changing ``sigma`` in place
    between forward and backward is an error (torch's version check).
    """

    @staticmethod
    def forward(ctx, f, sigma, plan, G, opts):
        opts = dict(opts or {})
        _bind(plan, sigma)
        u, st = plan.solve(f.detach(), None if G is None else G.detach(), **opts)
        ctx.plan, ctx.opts, ctx.stats = plan, opts, st
        ctx.has_sigma = sigma is not None
        if sigma is not None:
            ctx.save_for_backward(u, sigma)
        else:
            ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        saved = ctx.saved_tensors
        u = saved[0]
        sigma = saved[1] if ctx.has_sigma else None
        plan = ctx.plan
        _bind(plan, sigma)
        lam, _ = plan.adjoint(grad_u.detach().contiguous(), **ctx.opts)
        grad_f = lam if ctx.needs_input_grad[0] else None
        grad_sigma = None
        if ctx.has_sigma and ctx.needs_input_grad[1]:
            grad_sigma = plan.coeff_grad(u, lam)
        return grad_f, grad_sigma, None, None, None


def solve(f, sigma, plan, G=None, **opts):
    """Differentiable solve with respect to f and sigma."""
    return SGMLSolve.apply(f, sigma, plan, G, opts)
