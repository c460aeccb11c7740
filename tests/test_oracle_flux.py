"""Pins of the oracle's flux, ghost-state and block-solve pieces against the
mathematics they restate (paper Sec. 1 and Sec. 2.1: physical flux,
Remark on numerical fluxes, Remark on boundary conditions)."""
import math

import numpy as np
import pytest

import oracle
from paper_1608_06721_amd import workloads as W

G = 9.81
EPS_R = 0.03


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def swe_flux(axis, h, u, v):
    """Flux of the shallow water equations (Sec. 1): x-direction
    (hu, hu^2 + g h^2/2, huv), y-direction (hv, huv, hv^2 + g h^2/2)."""
    if axis == 0:
        return np.array([h * u, h * u * u + G * h * h / 2, h * u * v])
    return np.array([h * v, h * u * v, h * v * v + G * h * h / 2])


@pytest.mark.parametrize("axis", [0, 1])
def test_physical_flux_is_the_swe_flux(axis):
    r = rng(1)
    for _ in range(50):
        h, u, v = r.uniform(0, 3), r.uniform(-2, 2), r.uniform(-2, 2)
        np.testing.assert_allclose(oracle.phys_flux(3, axis, G, h, u, v), swe_flux(axis, h, u, v),
                                   rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(oracle.phys_flux(2, 0, G, 1.3, 0.7, 0.0), swe_flux(0, 1.3, 0.7, 0)[:2],
                               rtol=1e-15)


@pytest.mark.parametrize("flux", [W.HLL, W.LLF, W.HLLC])
@pytest.mark.parametrize("axis", [0, 1])
def test_consistency(flux, axis):
    """F_hat(U, U) = F(U) (the consistency required of eq:totalFlux)."""
    r = rng(2)
    for _ in range(200):
        h, u, v = r.uniform(0, 3), r.uniform(-3, 3), r.uniform(-3, 3)
        got = oracle.num_flux(flux, 3, axis, G, EPS_R, h, u, v, h, u, v)
        ref = swe_flux(axis, h, u, v)
        np.testing.assert_allclose(got, ref, rtol=4e-15, atol=4e-15 * (1 + np.abs(ref).max()))


@pytest.mark.parametrize("flux", [W.HLL, W.LLF, W.HLLC])
def test_rotation_invariance(flux):
    """The y-flux of (h, u, v) is the x-flux of (h, v, u) with the momentum
    components swapped (rotational invariance of the SWE)."""
    r = rng(3)
    for _ in range(100):
        hL, uL, vL, hR, uR, vR = r.uniform(0, 2), *r.uniform(-2, 2, 2), r.uniform(0, 2), *r.uniform(-2, 2, 2)
        fy = oracle.num_flux(flux, 3, 1, G, EPS_R, hL, uL, vL, hR, uR, vR)
        fx = oracle.num_flux(flux, 3, 0, G, EPS_R, hL, vL, uL, hR, vR, uR)
        np.testing.assert_allclose(fy, fx[[0, 2, 1]], rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("flux", [W.HLL, W.LLF, W.HLLC])
def test_mirror_symmetry(flux):
    """Reflecting x -> -x maps the face problem (L, R) to (mirror R,
    mirror L); the mass and tangential fluxes change sign, the normal
    momentum flux does not."""
    r = rng(4)
    for _ in range(200):
        hL, uL, vL, hR, uR, vR = r.uniform(0, 2), *r.uniform(-3, 3, 2), r.uniform(0, 2), *r.uniform(-3, 3, 2)
        if r.uniform() < 0.2:
            hL = 0.0
        f = oracle.num_flux(flux, 3, 0, G, EPS_R, hL, uL, vL, hR, uR, vR)
        m = oracle.num_flux(flux, 3, 0, G, EPS_R, hR, -uR, vR, hL, -uL, vL)
        np.testing.assert_allclose(m, [-f[0], f[1], -f[2]], rtol=1e-12, atol=1e-12)


def test_llf_values():
    """LLF on a depth jump at rest: mass flux -s/2 (hR - hL) with
    s = sqrt(g max h)(1 + eps_r); momentum = (p(hL) + p(hR))/2."""
    hL, hR = 0.4, 1.1
    s = math.sqrt(G * hR) + EPS_R * math.sqrt(G * hR)
    got = oracle.num_flux(W.LLF, 3, 0, G, EPS_R, hL, 0, 0, hR, 0, 0)
    np.testing.assert_allclose(got, [-0.5 * s * (hR - hL), 0.25 * G * (hL ** 2 + hR ** 2), 0.0],
                               rtol=1e-15)


def test_hll_upwinds_supercritical():
    """HLL returns the upwind physical flux when both waves move one way."""
    for (hL, uL, hR, uR) in [(1.0, 5.0, 0.8, 4.5), (0.5, -6.0, 0.7, -5.0)]:
        got = oracle.num_flux(W.HLL, 2, 0, G, EPS_R, hL, uL, 0, hR, uR, 0)
        up = (hL, uL) if uL > 0 else (hR, uR)
        np.testing.assert_allclose(got, swe_flux(0, up[0], up[1], 0)[:2], rtol=1e-15)


def test_hll_dry_side_speeds():
    """With a dry left side the HLL left speed is u_R - 2 sqrt(g h_R); for a
    right state at rest the mass flux is then -sL sR hR / (sR - sL)."""
    hR = 0.3
    sL = -2 * math.sqrt(G * hR)
    cs = math.sqrt(G * (math.sqrt(G * hR) / 2) ** 2 / G)
    sR = max(math.sqrt(G * hR), (0 + 0) / 2 + 0 - math.sqrt(G * hR) + cs)
    got = oracle.num_flux(W.HLL, 2, 0, G, EPS_R, 0.0, 0.0, 0, hR, 0.0, 0)
    assert got[0] == pytest.approx((-sL * 0 + sL * sR * hR) / (sR - sL), rel=1e-14)


@pytest.mark.parametrize("nc", [2, 3])
def test_solve_block(nc):
    r = rng(5)
    for _ in range(100):
        D = r.uniform(-1, 1, (nc, nc)) + 3 * np.eye(nc)
        b = r.uniform(-1, 1, nc)
        np.testing.assert_allclose(oracle.solve_block(D.ravel(), b), np.linalg.solve(D, b),
                                   rtol=1e-12, atol=1e-13)
    Z = np.zeros((nc, nc))
    Z[:, 0] = 1.0
    assert (oracle.solve_block(Z.ravel(), np.ones(nc)) == 0).all()


def test_inflow_celerity_is_the_positive_root():
    r = rng(6)
    for _ in range(200):
        K, gq = r.uniform(-5, 10), r.uniform(0.01, 60)
        c = oracle.inflow_celerity(K, gq)
        roots = np.roots([2.0, -K, 0.0, -gq])
        pos = [x.real for x in roots if abs(x.imag) < 1e-9 and x.real > 0]
        assert len(pos) == 1
        assert c == pytest.approx(pos[0], rel=1e-13)


def inv(un, h):
    return un + 2 * math.sqrt(G * h)


@pytest.mark.parametrize("f", [0, 1, 2, 3])
def test_ghost_walls(f):
    h, u, v = 0.7, 0.3, -0.2
    g = oracle.ghost(W.wall(W.REFLECT), f, G, 1e-6, h, u, v)
    if f < 2:
        assert tuple(g) == (h, -u, v)
    else:
        assert tuple(g) == (h, u, -v)
    s = oracle.ghost(W.wall(W.SLIP), f, G, 1e-6, h, u, v)
    assert tuple(s) == ((h, 0.0, v) if f < 2 else (h, u, 0.0))


def test_ghost_subcritical_inflow_discharge():
    """Subcritical inflow with prescribed discharge q on the west side: the
    ghost carries discharge q into the domain, the prescribed tangential
    velocity, and the interior's outgoing invariant u_n + 2 sqrt(g h)
    (u_n along the outward normal -x)."""
    h, u, v = 1.2, 0.5, 0.1
    q, ut = 1.3, 0.05
    hg, ug, vg = oracle.ghost(W.open_q(q, ut), 0, G, 1e-6, h, u, v)
    assert hg * ug == pytest.approx(q, rel=1e-14)
    assert vg == ut
    assert inv(-ug, hg) == pytest.approx(inv(-u, h), rel=1e-14)
    # the same on the south side (outward normal -y)
    hg, ug, vg = oracle.ghost(W.open_q(q), 2, G, 1e-6, h, v, u)
    assert hg * vg == pytest.approx(q, rel=1e-14) and ug == 0.0
    assert inv(-vg, hg) == pytest.approx(inv(-u, h), rel=1e-14)


def test_ghost_subcritical_outflow_depth():
    h, u, v = 0.9, 0.6, -0.1
    hg, ug, vg = oracle.ghost(W.open_h(1.0), 1, G, 1e-6, h, u, v)
    assert hg == 1.0 and vg == v
    assert inv(ug, hg) == pytest.approx(inv(u, h), rel=1e-14)


def test_ghost_supercritical():
    h, u = 0.2, 3.0                      # Froude number > 1
    assert tuple(oracle.ghost(W.open_h(1.0), 1, G, 1e-6, h, u, 0.0)) == (h, u, 0.0)
    side = (W.OPEN, 0.3, 1.5, 0.0)       # everything prescribed: supercritical inflow
    hg, ug, vg = oracle.ghost(side, 0, G, 1e-6, h, u, 0.0)
    assert (hg, ug, vg) == (0.3, 1.5 / 0.3, 0.0)


def test_hllc_tangential_upwinding():
    """HLLC keeps HLL's mass and normal momentum fluxes and carries the
    tangential velocity of the side the contact wave comes from."""
    r = rng(7)
    for _ in range(100):
        hL, hR = r.uniform(0.3, 2, 2)
        uL, uR = r.uniform(-0.5, 0.5, 2)        # subcritical: sL < 0 < sR
        vL, vR = r.uniform(-1, 1, 2)
        hll = oracle.num_flux(W.HLL, 3, 0, G, EPS_R, hL, uL, vL, hR, uR, vR)
        hllc = oracle.num_flux(W.HLLC, 3, 0, G, EPS_R, hL, uL, vL, hR, uR, vR)
        assert hllc[0] == hll[0] and hllc[1] == hll[1]
        ut = vL if hllc[0] >= 0 else vR       # contact moves with the mass flux
        assert hllc[2] == pytest.approx(ut * hllc[0], rel=1e-14, abs=1e-300)
