"""GPU parity: the HIP path (called through the C ABI) against the CPU
oracle on identical seeded inputs.

Every kernel evaluates the same FP64 expressions in the same order as the
oracle without contraction, so the bar is bit-for-bit equality of every
array (numeric equality: +0 == -0).  The only non-bitwise quantity is the
global sum of ||R_i||_1 (a tree reduction on the GPU, a sequential sum in
the oracle), compared to 1e-13 relative.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1608_06721_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-parity]", *a, flush=True)
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
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, what
    bad = ~((a == b) | (np.isnan(a) & np.isnan(b)))
    if bad.any():
        idx = np.argwhere(bad)[:5]
        diff = np.abs(a - b)[bad].max()
        raise AssertionError("%s: %d entries differ (max |diff| %.3e), first at %s: %r vs %r" % (
            what, bad.sum(), diff, idx.tolist(), a[tuple(idx[0])], b[tuple(idx[0])]))


WALLS = [W.wall(), W.wall(), W.wall(), W.wall()]
CHAN = [W.open_q(0.8, 0.0), W.open_h(1.1), W.wall(), W.wall(W.SLIP)]


def tiny(dim, nx, ny, seed, bc, flux, **kw):
    z, U = W.random_state(dim, nx, ny, seed)
    p = W.default_params(dim, flux=flux, **kw)
    prob = W.Problem("tiny%d" % seed, dim, nx, ny, 0.0, nx / 4.0, 0.0, ny / 4.0 if dim == 2 else 1.0,
                     bc, p, z, U)
    return prob


def problems():
    out = []
    for flux in (W.HLL, W.LLF):
        out.append(tiny(1, 16, 1, 1, CHAN, flux, n_levels=2))
        out.append(tiny(2, 8, 8, 2, WALLS, flux, n_levels=2))
        out.append(tiny(2, 24, 16, 3, CHAN, flux, n_levels=3))   # odd coarse width
    out.append(W.bump_1d(200))
    out.append(W.lake_island(64, n_levels=4))
    out.append(W.channel(64, 64, n_levels=4))
    out.append(W.dry_hill(64, 32, n_levels=3))
    out.append(tiny(2, 24, 16, 5, CHAN, W.HLLC, n_levels=3))
    out.append(W.transcritical_bump_2d(80, 32, n_levels=3))
    out.append(tiny(2, 13, 7, 6, CHAN, W.LLF, n_levels=0))   # odd by odd, ragged colour rows
    return out


PROBS = problems()


@pytest.mark.parametrize("k", range(len(PROBS)))
def test_residual_bitwise(nmg, k):
    prob = PROBS[k]
    say("residual", prob.name, prob.nx, prob.ny)
    ctx = nmg.Context.from_problem(prob)
    z, U = dev(prob.z), dev(prob.U0)
    R = torch.empty_like(U)
    tot = ctx.residual(z, U, R)
    Ro, toto = oracle.residual(prob, prob.U0)
    same(host(R), Ro, "R")
    assert tot == pytest.approx(toto, rel=1e-13, abs=1e-300)


@pytest.mark.parametrize("k", range(len(PROBS)))
def test_assembly_and_galerkin_bitwise(nmg, k):
    prob = PROBS[k]
    say("assemble", prob.name, prob.nx, prob.ny)
    ctx = nmg.Context.from_problem(prob)
    z, U = dev(prob.z), dev(prob.U0)
    R = torch.empty_like(U)
    tot = ctx.assemble_residual_jacobian(z, U, R)
    Ao, bo, toto = oracle.assemble(prob, prob.U0)
    A, b = ctx.get_system(0)
    same(host(A), Ao, "A level 0")
    same(host(b), bo, "b level 0")
    assert tot == pytest.approx(toto, rel=1e-13, abs=1e-300)
    for lev, Ah in enumerate(oracle.hierarchy(Ao, prob.params["n_levels"])):
        if lev == 0:
            continue
        A, _ = ctx.get_system(lev, want_b=False)
        same(host(A), Ah, "A level %d" % lev)


def random_case(dim, nx, ny, seed, nl):
    A, b = W.random_system(dim, nx, ny, seed)
    r = np.random.Generator(np.random.PCG64(seed + 100))
    x0 = r.uniform(-1, 1, b.shape)
    p = W.default_params(dim, n_levels=nl)
    bc = WALLS
    prob = W.Problem("rand", dim, nx, ny, 0, 1, 0, 1, bc, p, np.zeros((ny, nx)), np.zeros_like(b))
    return prob, A, b, x0


LIN = [(1, 32, 1, 1, 3), (2, 16, 12, 2, 2), (2, 24, 16, 3, 3), (2, 8, 8, 4, 1)]
# levels spanning several 32x16 tiles of the fused half-sweep pairs, ragged in
# both directions, with odd coarse dimensions
TILED = [(2, 160, 72, 8, 2), (2, 96, 40, 9, 3)]


@pytest.mark.parametrize("case", LIN)
@pytest.mark.parametrize("iters", [1, 3])
def test_sgs_bitwise(nmg, case, iters):
    prob, A, b, x0 = random_case(*case)
    say("sgs", case, iters)
    ctx = nmg.Context.from_problem(prob)
    ctx.load_system(dev(A), dev(b))
    x = dev(x0)
    ctx.sgs(x, iters)
    same(host(x), oracle.sgs(A, b, x0, iters, order=W.REDBLACK), "x after SGS")


@pytest.mark.parametrize("case", LIN + TILED)
@pytest.mark.parametrize("nus", [(2, 2, 10), (1, 0, 3), (0, 1, 2), (0, 0, 1), (3, 1, 0)])
@pytest.mark.parametrize("cycles", [1, 3])
@pytest.mark.parametrize("coarse_cells", ["4096", "0"])
@pytest.mark.parametrize("gamma", [1, 2])
@pytest.mark.parametrize("fuse", ["3", "2", "1"])
def test_vcycle_bitwise(nmg, case, nus, cycles, coarse_cells, gamma, fuse, monkeypatch):
    """coarse_cells: levels up to this many cells run in the single-workgroup
    coarse-cycle kernel ("0": every level launched on its own); gamma = 2 is
    the W-cycle; fuse: most half sweeps per launch on the launched coarse
    levels (3: pairs and triples, 2: pairs, 1: every half sweep on its own)."""
    prob, A, b, x0 = random_case(*case)
    say("vcycle", case, nus, cycles, coarse_cells, gamma, fuse)
    monkeypatch.setenv("NMG_COARSE_CELLS", coarse_cells)
    monkeypatch.setenv("NMG_FUSE", fuse)
    p = dict(prob.params, nu1=nus[0], nu2=nus[1], nu_coarse=nus[2], gamma=gamma)
    ctx = nmg.Context.from_problem(prob, **p)
    ctx.load_system(dev(A), dev(b))
    x = dev(x0)
    ctx.mg_vcycle(x, cycles)
    same(host(x), oracle.vcycles(A, b, x0, p, cycles), "x after V-cycles")


# Cycles whose first coarse-kernel level (32x32, 32x24, 30x20 over an odd
# 15x10; 1024 cells in 1D)
# lives in global memory with at most one slot per colour and thread: its
# runs of half sweeps, and the restriction that follows them, execute with
# the level's block rows in registers (COP_REGRUN); NMG_COARSE_REG=0 runs the
# same operations one by one.  nu1 = 0 leaves a restriction with no run
# before it, nu2 = 0 a level whose correction is fixed up at the end.
# The coarsest level's runs use two lanes per cell where it has at most 128
# cells per colour (16x16, 8x6, the odd 15x10, 14x10 and the odd-by-odd 11x9
# under register-run 28x20 and 22x18 levels) and one lane per cell beyond
# that or in 1D: 18x16 (144 per colour, below a launched 36x32 level) fits
# LDS only in FP32 and runs one lane per cell there, from global memory in
# FP64.  NMG_COARSE_SPLIT=0 runs one lane per cell everywhere.
REG = [(2, 64, 64, 5, 2), (2, 64, 48, 6, 3), (1, 2048, 1, 7, 2), (2, 120, 80, 10, 3),
       (2, 72, 64, 11, 2), (2, 56, 40, 12, 2), (2, 44, 36, 13, 2)]


@pytest.mark.parametrize("case", REG)
@pytest.mark.parametrize("nus", [(2, 2, 10), (1, 0, 3), (0, 1, 2)])
@pytest.mark.parametrize("gamma", [1, 2, 3])
@pytest.mark.parametrize("reg", ["1", "0"])
@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("split", ["1", "0"])
def test_vcycle_register_runs_bitwise(nmg, case, nus, gamma, reg, fp32, split, monkeypatch):
    prob, A, b, x0 = random_case(*case)
    say("vcycle register runs", case, nus, gamma, reg, fp32, split)
    monkeypatch.setenv("NMG_COARSE_CELLS", "1024")
    monkeypatch.setenv("NMG_COARSE_REG", reg)
    monkeypatch.setenv("NMG_COARSE_SPLIT", split)
    p = dict(prob.params, nu1=nus[0], nu2=nus[1], nu_coarse=nus[2], gamma=gamma,
             inner_fp32=fp32)
    ctx = nmg.Context.from_problem(prob, **p)
    ctx.load_system(dev(A), dev(b))
    x = dev(x0)
    ctx.mg_vcycle(x, 2)
    same(host(x), oracle.vcycles(A, b, x0, p, 2), "x after cycles")


@pytest.mark.parametrize("lanes", ["default", "1", "4", "16"])
@pytest.mark.parametrize("k", [0, 1, 3, 7, 8, 9, 10, 12])
def test_blu_sweep_bitwise(nmg, k, lanes, monkeypatch):
    """Lanes per cell of the BLU-SGS half sweep: 1, 4 (one per evaluation of
    the forward differences), 16 (one per face and evaluation; 4 in 1D) or
    the default choice by mesh size."""
    prob = PROBS[k]
    say("blu", prob.name, lanes)
    if lanes == "default":
        monkeypatch.delenv("NMG_BLU_LANES", raising=False)
    else:
        monkeypatch.setenv("NMG_BLU_LANES", lanes)
    ctx = nmg.Context.from_problem(prob)
    z, U = dev(prob.z), dev(prob.U0)
    ctx.blu_sweep(z, U)
    same(host(U), oracle.blu_sweep(prob, prob.U0), "U after BLU-SGS")


SOLVES = [
    (lambda: W.bump_1d(200), 1e-10, {}),
    (lambda: W.wetdry_1d(128, n_levels=5), 1e-10, {}),
    (lambda: W.lake_island(64, n_levels=4), 0.0, dict(max_newton=5)),
    (lambda: W.channel(64, 64, n_levels=4), 0.0, dict(max_newton=12)),
    (lambda: W.dry_hill(128, 64, n_levels=5), 1e-10, {}),
    (lambda: W.dry_hill(128, 64, n_levels=5, gamma=2), 1e-10, {}),
    (lambda: W.transcritical_bump_2d(80, 32, n_levels=3), 0.0, dict(max_newton=6)),
]


@pytest.mark.parametrize("k", range(len(SOLVES)))
def test_newton_solve_bitwise(nmg, k):
    mk, tol, over = SOLVES[k]
    prob = mk()
    prob = prob.with_params(**over)
    say("newton", prob.name, tol, over)
    ctx = nmg.Context.from_problem(prob)
    z, U = dev(prob.z), dev(prob.U0)
    st = ctx.newton_mg_solve(z, U, tol)
    Uo, sto = oracle.newton_solve(prob, tol=tol)
    say("  gpu", st["status"], st["newton_steps"], st["res_l1"], "oracle", sto["status"],
        sto["newton_steps"], sto["res_l1"])
    assert st["status"] == sto["status"]
    assert st["newton_steps"] == sto["newton_steps"]
    assert st["n_pinned"] == sto["n_pinned"]
    same(host(U), Uo, "U after the solve")
    np.testing.assert_allclose(st["res_hist"], sto["res_hist"], rtol=1e-12, atol=1e-300)


def test_status_codes(nmg):
    say("status codes")
    prob = W.channel(64, 64, n_levels=4)
    # invalid grid: 2^n_levels does not divide nx
    with pytest.raises(nmg.NMGError) as e:
        nmg.Context.from_problem(prob, n_levels=7)
    assert e.value.code == -1
    # NaN in the initial state
    ctx = nmg.Context.from_problem(prob)
    U0 = prob.U0.copy()
    U0[1, 10, 10] = np.nan
    z, U = dev(prob.z), dev(U0)
    st = ctx.newton_mg_solve(z, U, 1e-10)
    assert st["status"] == "ENONFINITE"
    # all dry: every cell isolated, R = 0, immediate convergence
    dry = W.lake_island(32, surface=-1.0, n_levels=3)
    ctx = nmg.Context.from_problem(dry)
    U = dev(dry.U0)
    st = ctx.newton_mg_solve(dev(dry.z), U, 1e-10)
    assert st["status"] == "OK" and st["newton_steps"] == 0 and st["n_pinned"] == 32 * 32
    assert st["res_l1"] == 0.0
    # one step only
    ctx = nmg.Context.from_problem(prob, max_newton=1)
    U = dev(prob.U0)
    st = ctx.newton_mg_solve(dev(prob.z), U, 1e-10)
    assert st["status"] == "NOT_CONVERGED" and st["newton_steps"] == 1


def test_lake_at_rest_gpu(nmg):
    """Well-balanced on the GPU: five forced steps keep the lake at rest."""
    prob = W.lake_island(256, n_levels=6, max_newton=5)
    say("lake at rest 256^2")
    ctx = nmg.Context.from_problem(prob)
    z, U = dev(prob.z), dev(prob.U0)
    st = ctx.newton_mg_solve(z, U, 0.0)
    Uh = host(U)
    wet = prob.U0[0] > 0
    assert st["newton_steps"] == 5
    assert np.abs(Uh[1:]).max() < 1e-13
    assert np.abs((Uh[0] + prob.z)[wet] - 0.5).max() < 1e3 * np.finfo(float).eps
    assert (Uh[:, ~wet] == 0).all()


BENCH = dict(n_levels=8)


def test_full_size_assembly_and_cycle(nmg):
    """The benchmark workload (1024 x 1024 channel, deep hierarchy): residual,
    assembly, all Galerkin levels and one V-cycle from zero, bit for bit."""
    prob = W.channel(1024, 1024, **BENCH)
    say("full size 1024^2 assembly")
    ctx = nmg.Context.from_problem(prob)
    z, U = dev(prob.z), dev(prob.U0)
    R = torch.empty_like(U)
    ctx.assemble_residual_jacobian(z, U, R)
    Ao, bo, _ = oracle.assemble(prob, prob.U0)
    same(host(R), oracle.residual(prob, prob.U0)[0], "R 1024^2")
    A, b = ctx.get_system(0)
    same(host(A), Ao, "A 1024^2")
    same(host(b), bo, "b 1024^2")
    del A
    say("full size 1024^2 V-cycle")
    x = torch.zeros_like(U)
    ctx.mg_vcycle(x, 1)
    xo = oracle.vcycles(Ao, bo, np.zeros_like(bo), prob.params, 1)
    same(host(x), xo, "dU after one V-cycle 1024^2")


def test_full_size_benchmark_cycles(nmg):
    """The benchmark's own configuration and launch path (1024 x 1024 channel,
    6 levels, W-cycle: streamed 1024x1024 and 512x512 levels, fused pairs and
    a triple on the launched coarse levels, one coarse-kernel launch per two
    32x32 visits with register-resident runs): assembly and two W-cycles from
    zero, bit for bit."""
    prob = W.channel(1024, 1024, n_levels=6, gamma=2, bump_width=(0.2, 0.8), mound_amp=0.8)
    say("full size 1024^2 benchmark W-cycles")
    ctx = nmg.Context.from_problem(prob)
    z, U = dev(prob.z), dev(prob.U0)
    ctx.assemble_residual_jacobian(z, U)
    Ao, bo, _ = oracle.assemble(prob, prob.U0)
    x = torch.zeros_like(U)
    ctx.mg_vcycle(x, 2)
    same(host(x), oracle.vcycles(Ao, bo, np.zeros_like(bo), prob.params, 2),
         "dU after two W-cycles 1024^2")


def test_vcycle_long_smoothing_bitwise(nmg, monkeypatch):
    """A smoothing call of more than 16 iterations on a launched level (here
    the coarsest, 40 iterations, no coarse kernel) is planned without fused
    launches; the result is unchanged."""
    prob, A, b, x0 = random_case(2, 96, 40, 9, 2)
    monkeypatch.setenv("NMG_COARSE_CELLS", "0")
    p = dict(prob.params, nu1=2, nu2=2, nu_coarse=40, gamma=2)
    ctx = nmg.Context.from_problem(prob, **p)
    ctx.load_system(dev(A), dev(b))
    x = dev(x0)
    ctx.mg_vcycle(x, 2)
    same(host(x), oracle.vcycles(A, b, x0, p, 2), "x after cycles with nu_coarse = 40")


# --- FP32 inner V-cycle (hierarchy and smoother in FP32, Newton in FP64) ---

@pytest.mark.parametrize("case", LIN + TILED)
@pytest.mark.parametrize("nus", [(2, 2, 10), (1, 0, 3)])
@pytest.mark.parametrize("coarse_cells", ["256", "0"])
@pytest.mark.parametrize("fuse", ["3", "1"])
def test_vcycle_fp32_bitwise(nmg, case, nus, coarse_cells, fuse, monkeypatch):
    """fuse 1: every launched level smoothed one half sweep per launch, so
    each restriction reads the residuals its last pre-smoothing half sweep
    wrote (level 0 does so with any fuse)."""
    prob, A, b, x0 = random_case(*case)
    say("vcycle fp32", case, nus, coarse_cells, fuse)
    monkeypatch.setenv("NMG_COARSE_CELLS", coarse_cells)
    monkeypatch.setenv("NMG_FUSE", fuse)
    p = dict(prob.params, nu1=nus[0], nu2=nus[1], nu_coarse=nus[2], inner_fp32=1)
    ctx = nmg.Context.from_problem(prob, **p)
    ctx.load_system(dev(A), dev(b))
    Ag, bg = ctx.get_system(0)
    same(host(Ag), A.astype(np.float32).astype(np.float64), "A rounded to FP32")
    x = dev(x0)
    ctx.mg_vcycle(x, 2)
    same(host(x), oracle.vcycles(A, b, x0, p, 2), "x after FP32 V-cycles")


@pytest.mark.parametrize("k", [0, 2, 3, 4])
def test_newton_solve_fp32_inner_bitwise(nmg, k):
    mk, tol, over = SOLVES[k]
    prob = mk().with_params(inner_fp32=1, **over)
    say("newton fp32-inner", prob.name, tol, over)
    ctx = nmg.Context.from_problem(prob)
    z, U = dev(prob.z), dev(prob.U0)
    st = ctx.newton_mg_solve(z, U, tol)
    Uo, sto = oracle.newton_solve(prob, tol=tol)
    say("  gpu", st["status"], st["newton_steps"], st["res_l1"], "oracle", sto["status"],
        sto["newton_steps"], sto["res_l1"])
    assert st["status"] == sto["status"] and st["newton_steps"] == sto["newton_steps"]
    same(host(U), Uo, "U after the FP32-inner solve")


def test_full_size_fp32_cycle(nmg):
    """1024 x 1024 channel, FP32 inner: assembly rounding and one V-cycle."""
    prob = W.channel(1024, 1024, n_levels=8, inner_fp32=1)
    say("full size 1024^2 fp32 V-cycle")
    ctx = nmg.Context.from_problem(prob)
    z, U = dev(prob.z), dev(prob.U0)
    ctx.assemble_residual_jacobian(z, U)
    Ao, bo, _ = oracle.assemble(prob, prob.U0)
    A, b = ctx.get_system(0)
    same(host(A), Ao.astype(np.float32).astype(np.float64), "A 1024^2 in FP32")
    same(host(b), bo.astype(np.float32).astype(np.float64), "b 1024^2 in FP32")
    del A
    x = torch.zeros_like(U)
    ctx.mg_vcycle(x, 1)
    same(host(x), oracle.vcycles(Ao, bo, np.zeros_like(bo), prob.params, 1), "dU FP32 1024^2")


STEP1 = [
    (lambda: W.bump_1d(200, n_levels=3), 0.01),
    (lambda: W.channel(64, 32, n_levels=3, mound_amp=0.3, gamma=2), 0.01),
    (lambda: W.wetdry_1d(128, n_levels=5), 0.05),
]


@pytest.mark.parametrize("k", range(len(STEP1)))
def test_newton_with_step1_bitwise(nmg, k):
    """Algorithm 1 with Step 1 (nested BLU-SGS initial guess, eps_p a
    fraction of the initial residual) against the oracle: same sweeps, same
    Newton steps, same state bit for bit."""
    mk, frac = STEP1[k]
    prob = mk()
    r0 = oracle.residual(prob, oracle.threshold(prob, prob.U0))[1]
    prob = prob.with_params(eps_p=frac * r0)
    say("step1", prob.name, prob.params["eps_p"])
    ctx = nmg.Context.from_problem(prob)
    U = dev(prob.U0)
    st = ctx.newton_mg_solve(dev(prob.z), U, 1e-10)
    Uo, so = oracle.newton_solve(prob, tol=1e-10)
    say("  gpu", st["status"], st["newton_steps"], st["init_sweeps"], "oracle", so["status"],
        so["newton_steps"], so["init_sweeps"])
    assert (st["status"], st["newton_steps"], st["init_sweeps"]) == \
        (so["status"], so["newton_steps"], so["init_sweeps"])
    assert st["init_sweeps"] > 0
    same(host(U), Uo, "U after Step 1 + Newton")


def test_timing_hook_counts_full_finest_sweeps(nmg):
    """The measurement hook: every recorded launch is a full finest-level half
    sweep (half the cells each), and the recorded time is positive and not
    above the solve's own wall time."""
    import time
    prob = W.channel(64, 64, n_levels=3, gamma=2)
    ctx = nmg.Context.from_problem(prob)
    ctx.timing_enable(True, 1000)
    U = dev(prob.U0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = ctx.newton_mg_solve(dev(prob.z), U, 1e-10)
    wall = time.perf_counter() - t0
    tm = ctx.timing_read()
    say("timing", st["newton_steps"], tm)
    assert tm["launches"] > 0
    assert tm["cells"] == tm["launches"] * (64 * 64 // 2)
    assert 0 < tm["ms"] <= 1e3 * wall
