"""Differentiable pressure projection on the staggered grid.

Forward: u_new = u - G p with p the solution of A p = D u (the projection step of Goda's
scheme, Sec. 2.2, Eq. 4, with p standing for minus the pressure change).  Without a
Dirichlet wall A is singular: then D u - mean(D u) is solved for the zero-mean p.
Backward: the pressure solve is linear and A is symmetric, so its vector-Jacobian product is
D^T applied to the solution of the adjoint system (A lam = g, with the same projection); the
gradient's own vector-Jacobian product is G^T.  Both run in the library's HIP kernels.
"""
from __future__ import annotations

import torch

from .solver import Solver


class PressureSolve(torch.autograd.Function):
    """p = A^+ D u (with D u - mean(D u) when A is singular) for face velocities (u, v)."""

    @staticmethod
    def forward(ctx, u, v, solver: Solver):
        ctx.solver = solver
        b = solver.div(u.contiguous(), v.contiguous())
        p, _ = solver.solve(b)
        return p

    @staticmethod
    def backward(ctx, gp):
        solver = ctx.solver
        lam, _ = solver.solve_adjoint(gp.contiguous())
        gu, gv = solver.div_adjoint(lam)
        return gu, gv, None


class MacGrad(torch.autograd.Function):
    """(gu, gv) = G p, the face gradient (zero on Neumann wall faces)."""

    @staticmethod
    def forward(ctx, p, solver: Solver):
        ctx.solver = solver
        return solver.grad(p.contiguous())

    @staticmethod
    def backward(ctx, ggu, ggv):
        return ctx.solver.grad_adjoint(ggu.contiguous(), ggv.contiguous()), None


def project(u, v, solver: Solver):
    """Divergence-free projection (u, v) -> (u - G p, v - G p) and the pressure p."""
    p = PressureSolve.apply(u, v, solver)
    gu, gv = MacGrad.apply(p, solver)
    return u - gu, v - gv, p
