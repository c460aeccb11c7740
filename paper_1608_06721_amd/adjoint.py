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



class BatchGradients:
    """Bed gradients of one objective per problem for a batch of steady
    problems of one parameter set.  The steady states come from one batched
    Newton multigrid solve (nmg.Batch: every instance bit for bit its own
    solve); for each instance that converged, the objective's adjoint solve
    and bed vector-Jacobian product run on that instance's own context and
    stream, all instances concurrently (one host thread each; the library
    calls release the interpreter).  Each gradient equals that of
    steady_state() on the same instance bit for bit.  The contexts and
    streams are made once, here; the first adjoint solve of each context
    allocates its transposed matrix and Krylov vectors."""

    def __init__(self, probs, tol=1e-10, adj_tol=1e-12, adj_cycles=400, krylov=30):
        self.probs = list(probs)
        self.tol, self.adj_tol, self.adj_cycles, self.krylov = tol, adj_tol, adj_cycles, krylov
        self.stream = torch.cuda.current_stream()
        self.batch = nmg.Batch(self.probs, stream=self.stream)
        self.streams = [torch.cuda.Stream() for _ in self.probs]      # default priority
        self.ctxs = [nmg.Context.from_problem(p, stream=s)
                     for p, s in zip(self.probs, self.streams)]

    def close(self):
        for c in self.ctxs:
            c.close()
        self.batch.close()

    def __call__(self, zs, U0s, objective):
        """objective(k, U_k, z_k): a scalar torch expression, differentiable
        in U_k and z_k.  Returns (statuses, states, gradients, adjoint
        cycles): gradients[k] = dObjective/dz of instance k, None where its
        steady solve did not converge."""
        import threading
        import time
        n = len(self.probs)
        Us = [u.detach().clone() for u in U0s]
        zd = [z.detach() for z in zs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = self.batch.newton_mg_solve(zd, Us, self.tol)
        statuses = [r["status"] for r in res]
        self.newton_steps = [r["newton_steps"] for r in res]
        t1 = time.perf_counter()            # the batch solve synchronized the stream
        grads, cycles = [None] * n, [0] * n
        jobs = []
        for k in range(n):
            if statuses[k] != "OK":
                continue
            U = Us[k].clone().requires_grad_(True)
            z = zd[k].clone().requires_grad_(True)
            gU, gz = torch.autograd.grad(objective(k, U, z), (U, z), allow_unused=True)
            jobs.append((k, gU.detach().contiguous(),
                         torch.zeros_like(z) if gz is None else gz.detach()))
        ready = torch.cuda.Event()
        ready.record(self.stream)
        errors = []

        def run(k, gU, gz):
            try:
                s, ctx = self.streams[k], self.ctxs[k]
                s.wait_event(ready)
                with torch.cuda.stream(s):
                    lam, cyc, rel = ctx.adjoint_solve(zd[k], Us[k], gU, tol=self.adj_tol,
                                                      max_cycles=self.adj_cycles,
                                                      krylov=self.krylov)
                    if cyc >= self.adj_cycles and rel > self.adj_tol:
                        raise nmg.NMGError(1, "adjoint solve reached %d cycles at relative "
                                              "residual %.3e" % (cyc, rel))
                    grads[k] = gz - ctx.bed_vjp(zd[k], Us[k], lam)
                    cycles[k] = cyc
            except Exception as e:          # reported after every thread has ended
                errors.append((k, e))

        threads = [threading.Thread(target=run, args=job) for job in jobs]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        for k, _, _ in jobs:
            self.stream.wait_stream(self.streams[k])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        self.last_seconds = dict(forward=t1 - t0, adjoint=t2 - t1)
        if errors:
            k, e = errors[0]
            raise RuntimeError("adjoint of instance %d failed: %s" % (k, e))
        return statuses, Us, grads, cycles
