"""The steady state as a differentiable function of the bed.

`steady_state(solver, z, U0)` returns the converged state U*(z) of
Algorithm 1 (the library's Newton multigrid solve); its backward pass is
the adjoint of the steady equations R(U*, z) = 0: for an upstream gradient
v = dL/dU*, it solves (dR/dU)^T lam = v with the library's multigrid on the
transposed Newton matrix and returns dL/dz = -(dR/dz)^T lam (the library's
bed vector-Jacobian product).  Every step runs in the HIP library; this
module only marshals tensors.
"""
from __future__ import annotations

import torch

from . import nmg


class SteadyState(torch.autograd.Function):
    @staticmethod
    def forward(ctx, z, U0, solver, tol, adj_tol, adj_cycles, krylov):
        U = U0.detach().clone()
        st = solver.newton_mg_solve(z.detach(), U, tol)
        if st["status"] != "OK":
            raise nmg.NMGError(1, "steady solve did not converge: %s" % st["status"])
        ctx.save_for_backward(z.detach(), U)
        ctx.solver, ctx.adj_tol, ctx.adj_cycles, ctx.krylov = solver, adj_tol, adj_cycles, krylov
        ctx.stats = st
        return U

    @staticmethod
    def backward(ctx, gU):
        z, U = ctx.saved_tensors
        lam, cycles, rel = ctx.solver.adjoint_solve(z, U, gU.contiguous(), tol=ctx.adj_tol,
                                                    max_cycles=ctx.adj_cycles, krylov=ctx.krylov)
        ctx.adjoint_cycles, ctx.adjoint_rel = cycles, rel
        if cycles >= ctx.adj_cycles and rel > ctx.adj_tol:
            raise nmg.NMGError(1, "adjoint solve reached %d cycles at relative residual %.3e"
                               % (cycles, rel))
        gz = -ctx.solver.bed_vjp(z, U, lam)
        return gz, None, None, None, None, None, None


def steady_state(solver, z, U0, tol=1e-10, adj_tol=1e-12, adj_cycles=400, krylov=30):
    """U*(z) from U0 with `solver` (an nmg.Context for the grid and BC),
    differentiable with respect to z; the backward pass solves the adjoint to
    a relative residual adj_tol with GMRES(krylov)-accelerated cycles
    (krylov = 0: plain cycles) within adj_cycles cycles."""
    return SteadyState.apply(z, U0, solver, tol, adj_tol, adj_cycles, krylov)


def gauge_misfit(U, z, gauges, target):
    """sum over gauge cells (flat indices) of (h + z - target)^2."""
    eta = (U[0] + z).reshape(-1)
    return ((eta[gauges] - target) ** 2).sum()
