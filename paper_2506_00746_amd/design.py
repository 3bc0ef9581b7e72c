"""PDE-constrained design on top of the C ABI: a ``torch.autograd.Function``
whose forward is the Newton-CG solve of R(u; rho) = 0 and whose backward is
the adjoint gradient (paper: the design paragraph after Eq. (3) -- adjoint
loads from quadrature-point derivatives instead of black-box AD).

``DesignSolve.apply(rho, problem, opts)`` returns u(rho).  For any scalar
Phi(u) built with torch, ``Phi.backward()`` calls the adjoint solve
J(u) lambda = M dPhi/du and returns dPhi/drho = -lambda^T dR/drho, which the
library computes by one per-element kernel (no G^T, B G u recomputed).
"""
from __future__ import annotations

import torch

from .feod import Problem


class DesignSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho: torch.Tensor, problem: Problem, opts: dict | None = None):
        opts = dict(opts or {})
        rho64 = rho.detach().to(device=problem.device, dtype=torch.float64).contiguous().clone()
        problem.set_rho(rho64)
        u, rep = problem.newton_solve(None, **opts)
        ctx.problem = problem
        ctx.opts = opts
        ctx.report = rep
        ctx.rho_meta = (rho.dtype, rho.device)
        # the problem's coefficient may be changed before backward runs (another
        # apply, set_rho): the gradient is taken at this call's rho
        ctx.save_for_backward(u, rho64)
        return u

    @staticmethod
    def backward(ctx, grad_u: torch.Tensor):
        u, rho64 = ctx.saved_tensors
        opts = {k: v for k, v in ctx.opts.items()
                if k in ("rtol", "max_cg", "check_every", "prec", "jacobi", "partial_assembly")}
        ctx.problem.set_rho(rho64)
        g_u = grad_u.to(device=u.device, dtype=torch.float64).contiguous()
        grad_rho, _, _ = ctx.problem.adjoint_gradient(u, g_u, **opts)
        dtype, device = ctx.rho_meta
        return grad_rho.to(device=device, dtype=dtype), None, None
