"""Pins of the oracle's sensitivity routines (the adjoint extension of the
steady solve): the block transpose is the matrix transpose, the bed
derivative of the residual is the derivative of eq:Res (brute-force and
central differences), multigrid solves the transposed system, and the
adjoint gradient of a gauge objective equals central differences of the
objective through full Newton solves."""
import numpy as np
import pytest

import oracle
from blockmat import dense, unvec, vec
from paper_1608_06721_amd import workloads as W


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.mark.parametrize("dim,nx,ny", [(1, 8, 1), (2, 6, 4), (2, 8, 8)])
def test_transpose_is_the_matrix_transpose(dim, nx, ny):
    A, _ = W.random_system(dim, nx, ny, seed=31)
    At = oracle.transpose_blocks(A)
    np.testing.assert_array_equal(dense(At), dense(A).T)


def wet_problem(nx=10, ny=6, seed=5):
    """A wet random state with open and wall sides (all faces active)."""
    z, U = W.random_state(2, nx, ny, seed)
    p = W.Problem("wet", 2, nx, ny, 0.0, 2.0, 0.0, 1.0,
                  [W.open_q(0.8, 0.0), W.open_h(1.1), W.wall(), W.wall(W.SLIP)],
                  W.default_params(2, n_levels=1), z, U)
    return p, U


def dry_problem():
    """The channel's lake at rest over emergent mounds: isolated cells and
    exactly dry cells next to wet ones."""
    p = W.channel(16, 8, n_levels=1, mound_amp=1.6)
    assert (p.U0[0] == 0).any()
    return p, p.U0.copy()


def dense_bed_derivative(prob, U, step, central=False):
    """d vec(R) / dz by differences of the whole residual, rows pinned as in
    the assembly."""
    z0 = prob.z
    N = prob.nx * prob.ny
    R0, _ = oracle.residual(prob, U)
    iso = oracle.isolated(prob, U).ravel()
    dry = (U[0].ravel() == 0.0) & bool(prob.params["dry_pin"])
    M = np.zeros((prob.nc * N, N))
    for j in range(N):
        zp = z0.copy().ravel()
        zp[j] += step
        Rp, _ = oracle.residual(W.dataclasses.replace(prob, z=zp.reshape(z0.shape)), U)
        if central:
            zm = z0.copy().ravel()
            zm[j] -= step
            Rm, _ = oracle.residual(W.dataclasses.replace(prob, z=zm.reshape(z0.shape)), U)
            d = (Rp - Rm) / (2 * step)
        else:
            d = (Rp - R0) / step
        d = d.reshape(prob.nc, N)
        d[:, iso] = 0.0
        d[1:, dry & ~iso] = 0.0
        M[:, j] = d.T.ravel()          # cell-major rows, as vec()
    return M


@pytest.mark.parametrize("mk", [wet_problem, dry_problem])
def test_bed_vjp_is_the_transposed_residual_difference(mk):
    prob, U = mk()
    lam = rng(7).uniform(-1, 1, U.shape)
    M = dense_bed_derivative(prob, U, prob.params["fd_eps"])
    ref = (M.T @ vec(lam)).reshape(prob.ny, prob.nx)
    got = oracle.bed_vjp(prob, U, lam)
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-6 * np.abs(ref).max())


def test_bed_vjp_is_the_bed_derivative():
    prob, U = wet_problem(seed=9)
    lam = rng(8).uniform(-1, 1, U.shape)
    M = dense_bed_derivative(prob, U, 1e-5, central=True)
    ref = (M.T @ vec(lam)).reshape(prob.ny, prob.nx)
    got = oracle.bed_vjp(prob, U, lam)
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-5 * np.abs(ref).max())


def test_multigrid_solves_the_adjoint_system():
    prob, U = wet_problem(16, 16, seed=3)
    prob = prob.with_params(n_levels=2)
    A, _, _ = oracle.assemble(prob, U)
    At = oracle.transpose_blocks(A)
    g = rng(4).uniform(-1, 1, U.shape)
    ref = np.linalg.solve(dense(At), vec(g))
    x = np.zeros_like(g)
    p = dict(prob.params, gamma=2)
    for _ in range(40):
        x = oracle.vcycles(At, g, x, p, 1)
    assert np.abs(vec(x) - ref).max() < 1e-9 * np.abs(ref).max()


def smooth_cells(z, gap, candidates):
    """Candidates whose bed differs from every neighbour's by more than
    `gap`.  The reconstruction's max(z_i, z_j) makes the residual only
    piecewise smooth in z, with a kink where two neighbouring beds are equal;
    a difference quotient with step d is a derivative only where no bed
    within the stencil is closer than d."""
    ny, nx = z.shape
    out = []
    for k in candidates:
        j, i = divmod(int(k), nx)
        nb = [z[jj, ii] for jj, ii in ((j, i - 1), (j, i + 1), (j - 1, i), (j + 1, i))
              if 0 <= ii < nx and 0 <= jj < ny]
        if min(abs(z[j, i] - v) for v in nb) > gap and int(k) not in out:
            out.append(int(k))
    return out


def steady(prob, U0, tol=5e-13):
    U, st = oracle.newton_solve(prob.with_params(max_newton=60), U0=U0, tol=tol)
    assert st["status"] == "OK", st
    return U


def test_adjoint_gradient_equals_central_differences():
    """J(z) = sum over gauges of (h + z - target)^2 at the steady state of a
    small channel with submerged mounds; dJ/dz = J_z - (dR/dz)^T lam with
    A^T lam = J_U against (J(z + d e_k) - J(z - d e_k)) / (2 d), d = 1e-6."""
    prob = W.channel(16, 8, n_levels=2, mound_amp=0.3)
    U = steady(prob, prob.U0)
    N = prob.nx * prob.ny
    r = rng(11)
    gauges = r.choice(N, 6, replace=False)
    eta = (U[0] + prob.z).ravel()
    target = eta[gauges] + r.uniform(-0.02, 0.02, gauges.size)

    def J(Uz, z):
        e = (Uz[0] + z).ravel()[gauges]
        return float(((e - target) ** 2).sum())

    w = np.zeros(N)
    w[gauges] = 2 * (eta[gauges] - target)
    JU = np.zeros_like(U)
    JU[0] = w.reshape(prob.ny, prob.nx)
    A, _, _ = oracle.assemble(prob, U)
    lam = unvec(np.linalg.solve(dense(oracle.transpose_blocks(A)), vec(JU)), prob.nc,
                prob.ny, prob.nx)
    grad = w.reshape(prob.ny, prob.nx) - oracle.bed_vjp(prob, U, lam)
    scale = np.abs(grad).max()
    d = 1e-6
    cells = smooth_cells(prob.z, 100 * d, list(gauges) + list(np.argsort(-np.abs(grad).ravel())))[:6]
    assert len(cells) >= 4
    for k in cells:
        zp = prob.z.copy().ravel(); zp[k] += d
        zm = prob.z.copy().ravel(); zm[k] -= d
        pp = W.dataclasses.replace(prob, z=zp.reshape(prob.z.shape))
        pm = W.dataclasses.replace(prob, z=zm.reshape(prob.z.shape))
        fd = (J(steady(pp, U), pp.z) - J(steady(pm, U), pm.z)) / (2 * d)
        g = grad.ravel()[k]
        assert abs(fd - g) <= 1e-5 * max(abs(fd), 1e-2 * scale), (k, fd, g)
