"""Seeded synthetic workloads: grids, bed topographies, boundary conditions,
initial states and method parameters.

This module holds input data only (no step of the method's arithmetic), so
that the GPU path and the CPU oracle are fed from the same place.  Every
array is float64 and generated on the host with numpy's PCG64 generator.

Layouts: cell vectors are component-major ``[nc][ny][nx]`` (x fastest); the
bed ``z`` is ``[ny][nx]``.  In 1D ``ny == 1`` and ``nc == 2`` (h, hu); in 2D
``nc == 3`` (h, hu, hv).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

REFLECT, SLIP, OPEN = 0, 1, 2
HLL, LLF, HLLC = 0, 1, 2
REDBLACK, LEX = 0, 1
NAN = float("nan")

# Side order W, E, S, N.  Each side: (kind, h, qn, ut); NaN = not prescribed.
Side = Tuple[int, float, float, float]


def default_params(dim: int, **kw) -> dict:
    """Method parameters with the paper's values (Sec. 3 preamble): eps=1e-8,
    alpha=3, tau=1, N_mg=2 (1D) / 3 (2D), h_eps=1e-6, eps_r=0.03; V(2,2),
    N_L=3; HLL in 1D, LLF in 2D.  dry_pin and pos_theta are the two
    wet/dry safeguards of this implementation (dry-cell momentum pin and the
    positivity-limited per-cell relaxation); dry_pin=0, pos_theta=0 gives
    the method exactly as printed.  eps_p > 0 turns on Step 1 of Algorithm 1
    (nested BLU-SGS initial guess) with that tolerance."""
    p = dict(flux=HLL if dim == 1 else LLF, g=9.81, alpha=3.0, fd_eps=1e-8, tau=1.0,
             h_eps=1e-6, eps_r=0.03, n_levels=3, nu1=2, nu2=2, nu_coarse=10,
             n_mg=2 if dim == 1 else 3, blu_sweeps=1, max_newton=500, order=REDBLACK,
             dry_pin=1, pos_theta=0.9 if dim == 2 else 0.0, inner_fp32=0, gamma=1,
             eps_p=0.0, init_max_sweeps=1000)
    for k, v in kw.items():
        if k not in p:
            raise KeyError(k)
        p[k] = v
    return p


@dataclasses.dataclass
class Problem:
    name: str
    dim: int
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float
    bc: List[Side]
    params: dict
    z: np.ndarray
    U0: np.ndarray

    @property
    def nc(self) -> int:
        return 2 if self.dim == 1 else 3

    @property
    def nb(self) -> int:
        return 3 if self.dim == 1 else 5

    def with_params(self, **kw) -> "Problem":
        p = dict(self.params)
        p.update(kw)
        return dataclasses.replace(self, params=p)


def cell_centres(x0, x1, n):
    dx = (x1 - x0) / n
    return x0 + (np.arange(n) + 0.5) * dx


def wall(kind=REFLECT) -> Side:
    return (kind, NAN, NAN, NAN)


def open_q(qn: float, ut: float = NAN) -> Side:
    return (OPEN, NAN, float(qn), ut)


def open_h(h: float) -> Side:
    return (OPEN, float(h), NAN, NAN)


def bump_z(x):
    """Bed of the 1D transcritical/wet-dry examples: 0.2 - 0.05 (x-10)^2 on
    8 < x < 12, else 0."""
    return np.where((x > 8.0) & (x < 12.0), 0.2 - 0.05 * (x - 10.0) ** 2, 0.0)


def bump_1d(n: int = 200, **kw) -> Problem:
    """1D subcritical flow over a bump: [0, 25], inflow discharge 4.42,
    outflow depth 2, start h + z = 2, hu = 4.42, HLL."""
    x = cell_centres(0.0, 25.0, n)
    z = bump_z(x)[None, :]
    U0 = np.zeros((2, 1, n))
    U0[0, 0] = 2.0 - z[0]
    U0[1, 0] = 4.42
    bc = [open_q(4.42), open_h(2.0), wall(), wall()]
    return Problem("bump_1d_%d" % n, 1, n, 1, 0.0, 25.0, 0.0, 1.0, bc,
                   default_params(1, **kw), z, U0)


def smooth_1d(n: int = 256, **kw) -> Problem:
    """Smooth subcritical 1D flow (Example 3.1 set-up): [-10, 10], bed
    0.2 exp(-(x+1)^2/2) + 0.3 exp(-(x-1.5)^2), discharge 1 imposed upstream,
    depth 1 imposed downstream; start h = 1 - z, hu = 1."""
    x = cell_centres(-10.0, 10.0, n)
    z = (0.2 * np.exp(-((x + 1.0) ** 2) / 2.0) + 0.3 * np.exp(-((x - 1.5) ** 2)))[None, :]
    U0 = np.zeros((2, 1, n))
    U0[0, 0] = 1.0 - z[0]
    U0[1, 0] = 1.0
    bc = [open_q(1.0), open_h(1.0), wall(), wall()]
    return Problem("smooth_1d_%d" % n, 1, n, 1, -10.0, 10.0, 0.0, 1.0, bc,
                   default_params(1, **kw), z, U0)


def wetdry_1d(n: int = 512, **kw) -> Problem:
    """1D lake at rest with an emerged bump (Example 3.3 set-up): bed as
    bump_z on [0, 20], start h = max(0.22 - z, 0) at rest, depth 0.1 imposed
    at both ends, LLF.  Steady state: h = max(0.1 - z, 0), u = 0."""
    x = cell_centres(0.0, 20.0, n)
    z = bump_z(x)[None, :]
    U0 = np.zeros((2, 1, n))
    U0[0, 0] = np.maximum(0.22 - z[0], 0.0)
    bc = [open_h(0.1), open_h(0.1), wall(), wall()]
    kw.setdefault("flux", LLF)
    return Problem("wetdry_1d_%d" % n, 1, n, 1, 0.0, 20.0, 0.0, 1.0, bc,
                   default_params(1, **kw), z, U0)


def lake_island(n: int = 256, surface: float = 0.5, **kw) -> Problem:
    """2D lake at rest with a dry island: [0,1]^2, z = 0.8 exp(-50 r^2) about
    (0.5, 0.5), h = max(0, surface - z), u = v = 0, reflective walls, LLF."""
    x = cell_centres(0.0, 1.0, n)
    y = cell_centres(0.0, 1.0, n)
    X, Y = np.meshgrid(x, y)
    z = 0.8 * np.exp(-50.0 * ((X - 0.5) ** 2 + (Y - 0.5) ** 2))
    U0 = np.zeros((3, n, n))
    U0[0] = np.maximum(0.0, surface - z)
    bc = [wall(), wall(), wall(), wall()]
    return Problem("lake_island_%d" % n, 2, n, n, 0.0, 1.0, 0.0, 1.0, bc,
                   default_params(2, **kw), z, U0)


CHANNEL_SEED = 160806721


def channel_bed(nx: int, ny: int, seed: int = CHANNEL_SEED, lx: float = 10.0, ly: float = 2.0,
                n_bumps: int = 16, n_mounds: int = 2, max_background: float = 0.45,
                mound_amp: float = 1.6, mound_width: float = 0.25,
                bump_width=(0.05, 0.4), bump_amp=(0.0, 0.3)):
    """Bed of the 2D channel workload: 16 seeded Gaussians (amplitude
    U[0, 0.3], width U[0.05, 0.4], centre uniform in the channel), redrawn
    until their sum stays below 0.45 on the grid (keeps the flow
    subcritical), plus two emergent mounds of amplitude 1.6 and width 0.25
    with centres in [3, 7] x [0.5, 1.5] at least 1 apart."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = cell_centres(0.0, lx, nx)
    y = cell_centres(0.0, ly, ny)
    X, Y = np.meshgrid(x, y)
    for _ in range(1000):
        amp = rng.uniform(bump_amp[0], bump_amp[1], n_bumps)
        wid = rng.uniform(bump_width[0], bump_width[1], n_bumps)
        cx = rng.uniform(0.0, lx, n_bumps)
        cy = rng.uniform(0.0, ly, n_bumps)
        zb = np.zeros_like(X)
        for k in range(n_bumps):
            zb += amp[k] * np.exp(-((X - cx[k]) ** 2 + (Y - cy[k]) ** 2) / wid[k] ** 2)
        if zb.max() <= max_background:
            break
    else:
        raise RuntimeError("no admissible background bed")
    centres = []
    while len(centres) < n_mounds:
        c = (rng.uniform(3.0, 7.0), rng.uniform(0.5, 1.5))
        if all(math.hypot(c[0] - d[0], c[1] - d[1]) >= 1.0 for d in centres):
            centres.append(c)
    z = zb.copy()
    for (mx, my) in centres:
        z += mound_amp * np.exp(-((X - mx) ** 2 + (Y - my) ** 2) / mound_width ** 2)
    return z


def channel(nx: int = 1024, ny: int = 1024, seed: int = CHANNEL_SEED, qn: float = 1.0,
            h_out: float = 1.0, mound_amp: float = 1.6, mound_width: float = 0.25,
            bump_width=(0.05, 0.4), bump_amp=(0.0, 0.3), **kw) -> Problem:
    """2D steady channel flow on [0,10] x [0,2]: inflow discharge qn (no
    tangential velocity) at x = 0, outflow depth h_out at x = 10, reflective
    walls at y = 0 and y = 2; start from the lake at rest
    (max(0, h_out - z), 0, 0); LLF."""
    z = channel_bed(nx, ny, seed, mound_amp=mound_amp, mound_width=mound_width,
                    bump_width=bump_width, bump_amp=bump_amp)
    U0 = np.zeros((3, ny, nx))
    U0[0] = np.maximum(0.0, h_out - z)
    bc = [open_q(qn, 0.0), open_h(h_out), wall(), wall()]
    return Problem("channel_%dx%d_s%d" % (nx, ny, seed), 2, nx, ny, 0.0, 10.0, 0.0, 2.0, bc,
                   default_params(2, **kw), z, U0)


# Bed of the measured 1024 x 1024 channel solve: the configured 16 bumps
# (amplitude U[0, 0.3], width U[0.05, 0.4]) and two emergent mounds of
# amplitude 1.1 and width 0.5.  Mounds of amplitude 1.6 and width 0.25 (the
# channel() default) give no steady state the method reaches.
BENCH_BED = dict(bump_width=(0.05, 0.4), mound_amp=1.1, mound_width=0.5)
# The bed measured before, kept as a second workload: wide bumps (width
# U[0.2, 0.8]) and mounds of amplitude 0.8, of which one emerges.
ONE_ISLAND_BED = dict(bump_width=(0.2, 0.8), mound_amp=0.8, mound_width=0.25)


def benchmark_channel(n: int = 1024, bed: dict = None, **kw) -> Problem:
    """The measured steady channel solve at n x n: bed BENCH_BED (or `bed`),
    Algorithm 1 with Step 1 (eps_p = 0.2, the value of the paper's
    experiments), W(2,2) cycles (gamma = 2) down to a 32 x 32 coarsest level,
    everything else as in channel()."""
    kw.setdefault("n_levels", int(round(math.log2(n))) - 5)
    kw.setdefault("gamma", 2)
    kw.setdefault("eps_p", 0.2)
    bed = dict(BENCH_BED if bed is None else bed)
    for k in list(bed):
        if k in kw:
            bed[k] = kw.pop(k)
    p = channel(n, n, **bed, **kw)
    p.name = "bench_channel_%d" % n
    return p


BATCH_SEED = CHANNEL_SEED + 1


def batch_channels(n: int = 64, sizes=(128, 256, 384, 512), q_range=(0.5, 2.0),
                   seed: int = BATCH_SEED, bump_width=(0.2, 0.8), mound_amp: float = 0.8,
                   **kw) -> list:
    """A batch of independent steady channel problems of uneven size: for
    instance k, nx and ny are drawn independently from `sizes`, the bed is
    channel_bed with seed + k, and the inflow discharge is drawn from
    U[q_range]; everything else (and every solver parameter in kw) as in
    channel()."""
    rng = np.random.Generator(np.random.PCG64(seed))
    probs = []
    for k in range(n):
        nx = int(rng.choice(sizes))
        ny = int(rng.choice(sizes))
        q = float(rng.uniform(*q_range))
        p = channel(nx, ny, seed=seed + k, qn=q, bump_width=bump_width, mound_amp=mound_amp, **kw)
        p.name = "batch%d_%dx%d_q%.3f" % (k, nx, ny, q)
        probs.append(p)
    return probs


ADJOINT_SEED = 160806821


@dataclasses.dataclass
class GaugeCase:
    """One topography of the gauge-misfit gradient workload: the problem,
    its gauge cells (flat indices) and the bed whose steady state defines the
    gauge targets."""
    prob: Problem
    gauges: np.ndarray
    z_true: np.ndarray


def gauge_cases(n: int = 16, size: int = 512, n_gauges: int = 64, seed: int = ADJOINT_SEED,
                bump_width=(0.2, 0.8), mound_amp: float = 0.8, **kw) -> list:
    """Topography b < n: the steady channel of channel() at size x size with
    bed seed `seed + b`; n_gauges gauge cells drawn without replacement among
    the cells wet (h > 0.05) in the initial lake at rest; the target bed adds
    0.02 exp(-r^2 / 0.3^2) around a seeded centre in [3, 7] x [0.5, 1.5]."""
    out = []
    for b in range(n):
        p = channel(size, size, seed=seed + b, bump_width=bump_width, mound_amp=mound_amp, **kw)
        rng = np.random.Generator(np.random.PCG64(seed + 1000 + b))
        wet = np.flatnonzero(p.U0[0].ravel() > 0.05)
        gauges = np.sort(rng.choice(wet, n_gauges, replace=False))
        cx, cy = rng.uniform(3.0, 7.0), rng.uniform(0.5, 1.5)
        X, Y = np.meshgrid(cell_centres(p.x0, p.x1, p.nx), cell_centres(p.y0, p.y1, p.ny))
        z_true = p.z + 0.02 * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / 0.3 ** 2)
        p.name = "gauges%d_%dx%d" % (b, size, size)
        out.append(GaugeCase(p, gauges, z_true))
    return out


def random_state(dim: int, nx: int, ny: int, seed: int, hmin=0.5, hmax=2.0, umax=0.5):
    """Smooth-ish random wet state (h in [hmin, hmax], |u|, |v| < umax) and
    bed in [0, 0.2], for unit tests of the discretization."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nc = 2 if dim == 1 else 3
    h = rng.uniform(hmin, hmax, (ny, nx))
    U = np.zeros((nc, ny, nx))
    U[0] = h
    U[1] = h * rng.uniform(-umax, umax, (ny, nx))
    if nc == 3:
        U[2] = h * rng.uniform(-umax, umax, (ny, nx))
    z = rng.uniform(0.0, 0.2, (ny, nx))
    return z, U


def random_system(dim: int, nx: int, ny: int, seed: int, diag_boost: float = 4.0):
    """Random block system (A in [nb][nc][nc][ny][nx] layout, b in
    [nc][ny][nx]) whose diagonal blocks dominate, for tests of the linear
    multigrid pieces on their own.  Off-diagonal blocks pointing out of the
    grid are zero."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nc = 2 if dim == 1 else 3
    nb = 3 if dim == 1 else 5
    A = rng.uniform(-1.0, 1.0, (nb, nc, nc, ny, nx))
    for r in range(nc):
        A[0, r, r] += diag_boost * nb
    A[1, :, :, :, 0] = 0.0
    A[2, :, :, :, nx - 1] = 0.0
    if dim == 2:
        A[3, :, :, 0, :] = 0.0
        A[4, :, :, ny - 1, :] = 0.0
    b = rng.uniform(-1.0, 1.0, (nc, ny, nx))
    return A, b


def dry_hill(nx: int = 128, ny: int = 64, **kw) -> Problem:
    """2D channel flow around a hill with a dry top (Example 3.7 set-up):
    [0, 25] x [-5, 5], z = 1.2 - 0.3 ((x-10)^2 + y^2) inside radius 2, else 0;
    discharge 0.1 at x = 0, depth 0.2 at x = 25, reflective walls at y = +-5;
    start h = max(0.2 - z, 0) at rest; LLF."""
    x = cell_centres(0.0, 25.0, nx)
    y = cell_centres(-5.0, 5.0, ny)
    X, Y = np.meshgrid(x, y)
    r2 = (X - 10.0) ** 2 + Y ** 2
    z = np.where(r2 < 4.0, 1.2 - 0.3 * r2, 0.0)
    U0 = np.zeros((3, ny, nx))
    U0[0] = np.maximum(0.2 - z, 0.0)
    bc = [open_q(0.1, 0.0), open_h(0.2), wall(), wall()]
    return Problem("dry_hill_%dx%d" % (nx, ny), 2, nx, ny, 0.0, 25.0, -5.0, 5.0, bc,
                   default_params(2, **kw), z, U0)


def transcritical_bump_2d(nx: int = 160, ny: int = 64, **kw) -> Problem:
    """2D flow over a bump (Example 3.6 set-up): [0, 25] x [-5, 5],
    z = 0.2 - 0.05 ((x-10)^2 + y^2) inside radius 2, discharge 1.53 at x = 0,
    depth 0.52 at x = 25, reflective walls at y = +-5, HLLC; start from rest
    at the outflow level, h = max(0.52 - z, 0)."""
    x = cell_centres(0.0, 25.0, nx)
    y = cell_centres(-5.0, 5.0, ny)
    X, Y = np.meshgrid(x, y)
    r2 = (X - 10.0) ** 2 + Y ** 2
    z = np.where(r2 < 4.0, 0.2 - 0.05 * r2, 0.0)
    U0 = np.zeros((3, ny, nx))
    U0[0] = np.maximum(0.52 - z, 0.0)
    bc = [open_q(1.53, 0.0), open_h(0.52), wall(), wall()]
    kw.setdefault("flux", HLLC)
    return Problem("bump2d_%dx%d" % (nx, ny), 2, nx, ny, 0.0, 25.0, -5.0, 5.0, bc,
                   default_params(2, **kw), z, U0)
