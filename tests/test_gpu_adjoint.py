"""GPU parity of the sensitivity path: the transposed Newton matrix and its
Galerkin levels, adjoint multigrid cycles and the bed vector-Jacobian
product bit for bit against the oracle; the converged adjoint against the
dense solve; the autograd gradient of a gauge misfit against the oracle's
adjoint gradient and against central differences of the objective through
GPU Newton solves (rel 1e-5)."""
import sys

import numpy as np
import pytest

import oracle
from blockmat import dense, unvec, vec
from paper_1608_06721_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-adjoint]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nmg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1608_06721_amd import nmg as _nmg
    _nmg.lib()
    return _nmg


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def same(a, b, what):
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape, what
    bad = ~((a == b) | (np.isnan(a) & np.isnan(b)))
    if bad.any():
        idx = np.argwhere(bad)[:3]
        raise AssertionError("%s: %d entries differ, first at %s: %r vs %r" % (
            what, bad.sum(), idx.tolist(), a[tuple(idx[0])], b[tuple(idx[0])]))


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def wet(nx, ny, seed, nl):
    z, U = W.random_state(2, nx, ny, seed)
    return W.Problem("wet", 2, nx, ny, 0.0, 2.0, 0.0, 1.0,
                     [W.open_q(0.8, 0.0), W.open_h(1.1), W.wall(), W.wall(W.SLIP)],
                     W.default_params(2, n_levels=nl), z, U), U


STATES = {
    "wet": lambda: wet(32, 16, 3, 2),
    "mounds": lambda: (lambda p: (p, p.U0.copy()))(W.channel(32, 16, n_levels=2, mound_amp=1.6)),
    "bump1d": lambda: (lambda p: (p, p.U0.copy()))(W.bump_1d(200).with_params(n_levels=3)),
}


@pytest.mark.parametrize("case", sorted(STATES))
def test_transposed_system_bitwise(nmg, case):
    prob, U = STATES[case]()
    say("transpose", case)
    ctx = nmg.Context.from_problem(prob)
    g = rng(1).uniform(-1, 1, U.shape)
    ctx.adjoint_solve(dev(prob.z), dev(U), dev(g), max_cycles=0)
    A, _, _ = oracle.assemble(prob, U)
    At = oracle.transpose_blocks(A)
    Ag, bg = ctx.get_system(0)
    same(host(Ag), At, "level-0 transposed blocks")
    same(host(bg), g, "adjoint right-hand side")
    Ag1, _ = ctx.get_system(1)
    same(host(Ag1), oracle.galerkin(At), "level-1 Galerkin of the transpose")


@pytest.mark.parametrize("case", sorted(STATES))
@pytest.mark.parametrize("gamma,cc", [(1, "1024"), (2, "1024"), (2, "0")])
def test_adjoint_cycles_bitwise(nmg, case, gamma, cc, monkeypatch):
    monkeypatch.setenv("NMG_COARSE_CELLS", cc)
    prob, U = STATES[case]()
    prob = prob.with_params(gamma=gamma)
    say("adjoint cycles", case, gamma, cc)
    ctx = nmg.Context.from_problem(prob)
    g = rng(2).uniform(-1, 1, U.shape)
    lam0 = rng(3).uniform(-0.1, 0.1, U.shape)
    A, _, _ = oracle.assemble(prob, U)
    At = oracle.transpose_blocks(A)
    for k in (1, 3):
        lam = dev(lam0)
        _, cyc, _ = ctx.adjoint_solve(dev(prob.z), dev(U), dev(g), lam=lam, tol=0.0, max_cycles=k)
        assert cyc == k
        same(host(lam), oracle.vcycles(At, g, lam0, prob.params, k), "lambda after %d cycles" % k)


@pytest.mark.parametrize("case", sorted(STATES))
def test_bed_vjp_bitwise(nmg, case):
    prob, U = STATES[case]()
    say("bed vjp", case)
    ctx = nmg.Context.from_problem(prob)
    lam = rng(4).uniform(-1, 1, U.shape)
    got = ctx.bed_vjp(dev(prob.z), dev(U), dev(lam))
    same(host(got), oracle.bed_vjp(prob, U, lam), "(dR/dz)^T lambda")


@pytest.mark.parametrize("krylov", [0, 30])
def test_adjoint_solve_converges_to_the_dense_solution(nmg, krylov):
    prob, U = wet(32, 16, 5, 2)
    ctx = nmg.Context.from_problem(prob, gamma=2)
    g = rng(5).uniform(-1, 1, U.shape)
    lam, cyc, rel = ctx.adjoint_solve(dev(prob.z), dev(U), dev(g), tol=1e-13, max_cycles=200,
                                      krylov=krylov)
    say("adjoint (krylov %d) converged in" % krylov, cyc, "cycles, rel", rel)
    assert rel <= 1e-13
    A, _, _ = oracle.assemble(prob, U)
    ref = unvec(np.linalg.solve(dense(oracle.transpose_blocks(A)), vec(g)), 3, 16, 32)
    np.testing.assert_allclose(host(lam), ref, rtol=0, atol=1e-10 * np.abs(ref).max())


def smooth_cells(z, gap, candidates):
    ny, nx = z.shape
    out = []
    for k in candidates:
        j, i = divmod(int(k), nx)
        nb = [z[jj, ii] for jj, ii in ((j, i - 1), (j, i + 1), (j - 1, i), (j + 1, i))
              if 0 <= ii < nx and 0 <= jj < ny]
        if min(abs(z[j, i] - v) for v in nb) > gap and int(k) not in out:
            out.append(int(k))
    return out


def test_autograd_gradient_matches_oracle_and_central_differences(nmg):
    from paper_1608_06721_amd import adjoint
    prob = W.channel(32, 16, n_levels=2, mound_amp=0.3, gamma=2)
    ctx = nmg.Context.from_problem(prob)
    N = prob.nx * prob.ny
    z = dev(prob.z).requires_grad_(True)
    U = adjoint.steady_state(ctx, z, dev(prob.U0), tol=5e-13)
    r = rng(6)
    gauges = torch.from_numpy(r.choice(N, 12, replace=False)).cuda()
    eta = (U[0] + z).detach().reshape(-1)[gauges]
    target = eta + torch.from_numpy(r.uniform(-0.02, 0.02, 12)).cuda()
    J = adjoint.gauge_misfit(U, z, gauges, target)
    J.backward()
    grad = host(z.grad)
    Us = host(U.detach())
    # the oracle's adjoint gradient at the same steady state (dense adjoint)
    gi = host(gauges)
    w = np.zeros(N)
    w[gi] = 2 * (host(eta) - host(target))
    JU = np.zeros_like(Us)
    JU[0] = w.reshape(prob.ny, prob.nx)
    A, _, _ = oracle.assemble(prob, Us)
    lam = unvec(np.linalg.solve(dense(oracle.transpose_blocks(A)), vec(JU)), 3, prob.ny, prob.nx)
    gref = w.reshape(prob.ny, prob.nx) - oracle.bed_vjp(prob, Us, lam)
    scale = np.abs(gref).max()
    np.testing.assert_allclose(grad, gref, rtol=0, atol=1e-8 * scale)
    # central differences of J through GPU Newton solves from the steady state
    d = 1e-6
    cells = smooth_cells(prob.z, 100 * d, list(gi) + list(np.argsort(-np.abs(grad).ravel())))[:6]
    say("fd cells", cells)

    def Jof(zz):
        Uz = dev(Us)
        st = ctx.newton_mg_solve(dev(zz), Uz, 5e-13)
        assert st["status"] == "OK", st
        e = (host(Uz)[0] + zz).ravel()[gi]
        return float(((e - host(target)) ** 2).sum())

    for k in cells:
        zp = prob.z.copy().ravel(); zp[k] += d
        zm = prob.z.copy().ravel(); zm[k] -= d
        fd = (Jof(zp.reshape(prob.z.shape)) - Jof(zm.reshape(prob.z.shape))) / (2 * d)
        g = grad.ravel()[k]
        say("  cell", k, "fd", fd, "adjoint", g)
        assert abs(fd - g) <= 1e-5 * max(abs(fd), 1e-2 * scale), (k, fd, g)


def test_full_size_gradient_spot_check(nmg):
    """One topography of the benchmark's gradient workload (512^2, 64 gauges,
    FP64 W-cycle) in its launch configuration: the autograd gradient against
    central differences (step 1e-6) through GPU Newton solves at the three
    largest-gradient cells whose bed is smooth at that step."""
    from paper_1608_06721_amd import adjoint
    case = W.gauge_cases(1, size=512, n_levels=5, gamma=2)[0]
    prob = case.prob
    ctx = nmg.Context.from_problem(prob)
    Ut = dev(prob.U0)
    assert ctx.newton_mg_solve(dev(case.z_true), Ut, 1e-10)["status"] == "OK"
    g = torch.from_numpy(case.gauges).cuda()
    target = (Ut[0] + dev(case.z_true)).reshape(-1)[g]
    z = dev(prob.z).requires_grad_(True)
    U = adjoint.steady_state(ctx, z, dev(prob.U0), tol=1e-11)
    J = adjoint.gauge_misfit(U, z, g, target)
    J.backward()
    grad = host(z.grad)
    Us = host(U.detach())
    scale = np.abs(grad).max()
    d = 1e-6
    cells = smooth_cells(prob.z, 100 * d, list(np.argsort(-np.abs(grad).ravel())[:200]))[:3]
    say("full size: |grad| max", scale, "cells", cells)
    assert len(cells) == 3
    tg = host(target)

    def Jof(zz):
        Uz = dev(Us)
        st = ctx.newton_mg_solve(dev(zz), Uz, 1e-11)
        assert st["status"] == "OK", st
        e = (host(Uz)[0] + zz).ravel()[case.gauges]
        return float(((e - tg) ** 2).sum())

    for k in cells:
        zp = prob.z.copy().ravel(); zp[k] += d
        zm = prob.z.copy().ravel(); zm[k] -= d
        fd = (Jof(zp.reshape(prob.z.shape)) - Jof(zm.reshape(prob.z.shape))) / (2 * d)
        gk = grad.ravel()[k]
        say("  cell", k, "fd", fd, "adjoint", gk)
        assert abs(fd - gk) <= 1e-5 * max(abs(fd), 1e-2 * scale), (k, fd, gk)


def test_batch_gradients_equal_single_gradients(nmg):
    """Batched bed gradients (one batched Newton solve of all topographies,
    then concurrent adjoint solves on per-topography contexts and streams)
    equal each topography's own autograd gradient bit for bit, with the same
    statuses; topographies without a steady state get no gradient."""
    from paper_1608_06721_amd import adjoint
    cases = W.gauge_cases(5, size=64, n_gauges=16, n_levels=3, gamma=2, max_newton=80)
    probs = [c.prob for c in cases]
    targets = []
    for c in cases:
        ctx = nmg.Context.from_problem(c.prob)
        Ut = dev(c.prob.U0)
        ctx.newton_mg_solve(dev(c.z_true), Ut, 1e-10)
        ctx.close()
        targets.append((Ut[0] + dev(c.z_true)).reshape(-1)[torch.from_numpy(c.gauges).cuda()])
    gauges = [torch.from_numpy(c.gauges).cuda() for c in cases]

    def objective(k, U, z):
        return adjoint.gauge_misfit(U, z, gauges[k], targets[k])

    bg = adjoint.BatchGradients(probs)
    try:
        zs = [dev(p.z) for p in probs]
        statuses, Us, grads, cycles = bg(zs, [dev(p.U0) for p in probs], objective)
    finally:
        bg.close()
    say("batch gradients", statuses, cycles)
    assert statuses.count("OK") >= 3
    for k, p in enumerate(probs):
        ctx = nmg.Context.from_problem(p)
        z = dev(p.z).requires_grad_(True)
        try:
            U = adjoint.steady_state(ctx, z, dev(p.U0))
        except nmg.NMGError:
            ctx.close()
            assert statuses[k] != "OK" and grads[k] is None
            continue
        assert statuses[k] == "OK"
        same(host(Us[k]), host(U.detach()), "steady state %d" % k)
        objective(k, U, z).backward()
        same(host(grads[k]), host(z.grad), "gradient %d" % k)
        ctx.close()
