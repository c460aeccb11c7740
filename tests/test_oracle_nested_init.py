"""Pins of Algorithm 1, Step 1 (nested BLU-SGS initial guess) in the oracle:
the definition replayed from the oracle's public pieces (child averages,
BLU-SGS sweeps until the level residual falls below eps_p 2^-l, injection),
the no-sweep limit, and Newton from the Step 1 guess reaching the same
steady state as Newton from the initial data."""
import numpy as np
import pytest

import oracle
from paper_1608_06721_amd import workloads as W


def avg2(a, dim):
    """One level of child averages in the order SW, SE, NW, NE."""
    if dim == 1:
        return (a[..., 0::2] + a[..., 1::2]) * 0.5
    return (((a[..., 0::2, 0::2] + a[..., 0::2, 1::2]) + a[..., 1::2, 0::2]) + a[..., 1::2, 1::2]) * 0.25


def inject(a, dim):
    return np.repeat(a, 2, axis=-1) if dim == 1 else np.repeat(np.repeat(a, 2, axis=-1), 2, axis=-2)


def coarse(prob, l, z_l):
    nx = prob.nx >> l
    ny = 1 if prob.dim == 1 else prob.ny >> l
    return W.dataclasses.replace(prob, nx=nx, ny=ny, z=z_l, U0=np.zeros((prob.nc, ny, nx)))


@pytest.mark.parametrize("mk", [lambda: W.bump_1d(200, n_levels=1),
                                lambda: W.channel(32, 16, n_levels=1, mound_amp=0.3)])
def test_one_level_definition(mk):
    prob = mk()
    U0 = oracle.threshold(prob, prob.U0)
    R0, r0 = oracle.residual(prob, U0)
    eps_p = 0.05 * r0
    p = dict(prob.params, eps_p=eps_p)
    got, sweeps = oracle.nested_init(prob, U0, params=p)
    k = sweeps[1]
    assert k >= 1
    z1 = avg2(prob.z, prob.dim)
    c = coarse(prob, 1, z1)
    U = avg2(U0, prob.dim)
    for s in range(k):
        assert oracle.residual(c, U, params=p)[1] >= eps_p / 2
        U = oracle.blu_sweep(c, U, params=p)
    assert oracle.residual(c, U, params=p)[1] < eps_p / 2
    np.testing.assert_array_equal(got, inject(U, prob.dim))


def test_no_sweeps_when_eps_p_is_large():
    prob = W.channel(32, 16, n_levels=3, mound_amp=0.3)
    U0 = oracle.threshold(prob, prob.U0)
    got, sweeps = oracle.nested_init(prob, U0, params=dict(prob.params, eps_p=1e30))
    assert sweeps == [0, 0, 0, 0]
    Uc = U0
    for _ in range(3):
        Uc = avg2(Uc, 2)
    for _ in range(3):
        Uc = inject(Uc, 2)
    np.testing.assert_array_equal(got, Uc)


def test_sweep_cap():
    prob = W.bump_1d(200, n_levels=2)
    _, sweeps = oracle.nested_init(prob, params=dict(prob.params, eps_p=1e-14, init_max_sweeps=3))
    assert sweeps == [0, 3, 3]


@pytest.mark.parametrize("mk", [lambda: W.bump_1d(200, n_levels=3),
                                lambda: W.channel(64, 32, n_levels=3, mound_amp=0.3, gamma=2)])
def test_newton_from_step1_reaches_the_same_steady_state(mk):
    prob = mk()
    U_a, st_a = oracle.newton_solve(prob, tol=1e-10)
    r0 = oracle.residual(prob, oracle.threshold(prob, prob.U0))[1]
    U_b, st_b = oracle.newton_solve(prob, tol=1e-10, params=dict(prob.params, eps_p=0.01 * r0))
    assert st_a["status"] == "OK" and st_b["status"] == "OK"
    assert st_b["init_sweeps"] > 0
    assert np.abs(U_a - U_b).max() < 1e-8
