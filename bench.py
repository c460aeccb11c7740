#!/usr/bin/env python3
"""Benchmark of the Newton multigrid steady shallow-water solver on one MI355X.

One step = one steady solve of the 2D channel workload (1024 x 1024 cells,
FP64, the bed of 16 seeded Gaussians and two emergent dry mounds): from the
resting initial state resident in HBM to sum_i ||R_i||_1 < tol, i.e. every
part of the hot path (Step 1's nested BLU-SGS initial guess, BLU-SGS
pre-smoothing, residual and FD-Jacobian assembly, Galerkin coarsening,
red-black block-SGS multigrid cycles, relaxed update) for as many Newton steps
as the solve needs.

Prints one JSON line with the metric, the roofline of the dominant kernel
(the finest-level block SGS half sweep, timed with hipEvents on the
library's stream), the time per phase of Algorithm 1, a roofline of the
whole Newton step, further workloads (the paper's default V-cycle, the FP32
inner cycle, the previously measured bed, the paper's 2D wet/dry example,
batched solves, bed gradients) and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "steady solves/s at 1024^2 to 1e-10 resid; SGS sweep HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of one 2D FP64 block SGS cell update: the 45 block
# entries (D and the four neighbour blocks), b_i, the new x_i, and the
# neighbours' x (each read once per half sweep, 24 B per update amortized).
SGS_BYTES_2D = 45 * 8 + 24 + 24 + 24
SGS_BYTES_2D_FP32 = 45 * 4 + 12 + 12 + 12
PHASES = ["step1", "blu", "assembly", "galerkin", "norm", "cycles", "update", "final"]


def sgs_source_digest():
    """sha256 (first 16 hex digits) of the sources the block SGS half-sweep
    kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for f in ("nmg_sgs.h", "nmg_internal.h"):
        h.update(open(os.path.join(HERE, "paper_1608_06721_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per finest-level SGS launch from the committed rocprofv3
    counter runs, or None if the kernel's sources changed since they were taken."""
    prof = os.path.join(HERE, "profiles", "sgs_halfsweep_channel1024_f64_pmc.md")
    try:
        fields = dict(l.split(":", 1) for l in open(prof).read().splitlines()
                      if l.startswith(("kernel_source_sha256_16:", "traffic_bytes_per_launch:")))
        digest = sgs_source_digest()
        if fields["kernel_source_sha256_16"].strip() != digest:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


# ---------------------------------------------------------------------------
# Algorithmic bytes of one Newton step (what the method must move between HBM
# and the chip if nothing stays cached), following the library's sequence of
# operations: Step 2.1 BLU-SGS, assembly, Galerkin levels, n_mg cycles of
# Algorithm 0 with the same-colour elision and zero starts, the update.

def newton_step_bytes(p, nx, ny, coarse_cells=1024, pair_cells=1 << 17):
    """Algorithmic HBM bytes of one Newton step of a 2D solve with parameters
    p on an nx x ny grid (per-unit byte counts in the comments)."""
    esz = 4 if p.get("inner_fp32", 0) else 8
    NL = int(p["n_levels"])
    N = [(nx >> l) * (ny >> l) for l in range(NL + 1)]
    blk = 45 * esz                     # one cell's five 3x3 blocks
    vec = 3 * esz                      # one cell's 3-vector in the hierarchy's type
    full = blk + 3 * vec               # half-sweep update reading every neighbour
    zero = 9 * esz + 2 * vec           # update after a zero start (D, b, write)
    lc = next((l for l in range(NL + 1) if N[l] <= coarse_cells), NL + 1)
    # levels whose last pre-smoothing half sweep writes its cells' residuals
    # for the restriction (launched one half sweep per launch)
    reuse = {l for l in range(NL) if l < lc and (l == 0 or N[l] > pair_cells)}
    st = [[1, 1] for _ in range(NL + 1)]        # 1: zero, 0: stored, 2: stored + pending
    last = [-1] * (NL + 1)
    tot = [0.0]

    def half(l, c, res=False):
        if last[l] == c:
            return
        mode_zero = st[l][c ^ 1] in (1, 3)
        n = N[l] / 2
        tot[0] += n * (zero if mode_zero else full) + (n * vec if res and not mode_zero else 0)
        if st[l][c ^ 1] >= 2:
            tot[0] += n * vec / 4           # the coarse correction read by prolongation
        st[l][c] = 0
        last[l] = c

    def smooth(l, iters, res_last=False):
        for it in range(iters):
            for q, c in enumerate((0, 1, 1, 0)):
                half(l, c, res_last and it == iters - 1 and q == 3)

    def materialize(l):
        for c in (0, 1):
            if st[l][c] == 1:
                tot[0] += N[l] / 2 * vec
            elif st[l][c] >= 2:
                tot[0] += N[l] / 2 * (2 * vec + vec / 4)
            st[l][c] = 0
            last[l] = -1

    def cycle(l):
        smooth(l, p["nu1"], l < NL and l in reuse)
        if l == NL:
            smooth(l, p["nu_coarse"])
        else:
            materialize(l)
            if l in reuse:          # half the residuals stored, the other half computed
                tot[0] += N[l] / 2 * vec + N[l] / 2 * (blk + 3 * vec) + N[l + 1] * vec
            else:
                tot[0] += N[l] * (blk + 3 * vec) + N[l + 1] * vec
            st[l + 1] = [1, 1]
            last[l + 1] = -1
            for _ in range(1 if l == 0 else int(p.get("gamma", 1))):
                cycle(l + 1)
            materialize(l + 1)
            st[l] = [3 if s == 1 else 2 for s in st[l]]
            last[l] = -1
        smooth(l, p["nu2"])

    for _ in range(int(p["n_mg"])):
        cycle(0)
    materialize(0)
    cyc = tot[0]
    n0 = N[0]
    blu = int(p["blu_sweeps"]) * 4 * (n0 / 2) * (32 + 24)   # own U, z and write per update
    copy = 2 * 24 * n0                                       # the kept iterate
    iso = (32 + 1) * n0
    assembly = n0 * (32 + vec + blk)
    galerkin = sum(N[l] * 5 * blk for l in range(1, NL + 1))
    update = n0 * (24 + vec + 24)
    return dict(total=blu + copy + iso + assembly + galerkin + cyc + update, cycles=cyc,
                blu=blu, assembly=assembly + iso, galerkin=galerkin, update=update + copy)


# ---------------------------------------------------------------------------

def phase_ms(ctx):
    ph = ctx.timing_phases()
    return {k: ph[k] for k in PHASES}


def timed_solves(ctx, z, U0, steps, warmup, tol, cap, label):
    """Warm-up solves, then `steps` timed solves from U0 (inputs resident in
    HBM); returns (seconds, stats, timing of the finest full SGS sweeps, phase
    times summed over the timed solves, the last solve's state)."""
    import torch
    for w in range(warmup):
        st = ctx.newton_mg_solve(z, U0.clone(), tol)
        print("[bench] %s warmup %d: %s steps=%d init=%d res=%.3e" % (
            label, w, st["status"], st["newton_steps"], st["init_sweeps"], st["res_l1"]),
            file=sys.stderr, flush=True)
    Us = [U0.clone() for _ in range(steps)]
    ctx.timing_enable(True, cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [ctx.newton_mg_solve(z, Us[k], tol) for k in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.timing_enable(False)
    for k, st in enumerate(stats):
        print("[bench] %s solve %d: %s steps=%d init=%d res=%.3e" % (
            label, k, st["status"], st["newton_steps"], st["init_sweeps"], st["res_l1"]),
            file=sys.stderr, flush=True)
    return dt, stats, ctx.timing_read(), phase_ms(ctx), Us[-1]


def sgs_roofline(tm, bytes_per_update, traffic=None):
    avg_ms = tm["ms"] / max(1, tm["launches"])
    cells = tm["cells"] / max(1, tm["launches"])
    bpl = cells * bytes_per_update
    achieved = bpl / (avg_ms * 1e-3) / 1e9 if tm["launches"] else None
    return dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                frac=(achieved / HBM_PEAK_GBS) if achieved else None,
                traffic=(traffic / (avg_ms * 1e-3) / 1e9) if (traffic and achieved) else None,
                traffic_bytes_per_launch=traffic, avg_launch_us=avg_ms * 1e3,
                launches=tm["launches"], bytes_per_launch=bpl)


def step_roofline(prob, phases, n_solves, n_newton):
    """Algorithmic bytes of one Newton step over the measured stream time of
    the Newton steps (phases blu..update, i.e. without Step 1 and the final
    residual), per step."""
    b = newton_step_bytes(prob.params, prob.nx, prob.ny)
    ms = sum(phases[k] for k in ("blu", "assembly", "galerkin", "norm", "cycles", "update"))
    ms_step = ms / max(1, n_solves * n_newton)
    ach = b["total"] / (ms_step * 1e-3) / 1e9 if ms_step > 0 else None
    return dict(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                frac=(ach / HBM_PEAK_GBS) if ach else None, bytes_per_newton_step=b["total"],
                bytes_by_part={k: v for k, v in b.items() if k != "total"},
                ms_per_newton_step=ms_step)


def describe_cycle(p):
    return "%s(%d,%d), N_L=%d, nu_coarse=%d, n_mg=%d" % (
        "V" if int(p.get("gamma", 1)) == 1 else "W", p["nu1"], p["nu2"], p["n_levels"],
        p["nu_coarse"], p["n_mg"])


def describe_bed(bed):
    return ("16 seeded Gaussians (amplitude U[0,0.3], width U[%g,%g]) + 2 mounds of amplitude "
            "%g, width %g (seed 160806721)" % (bed["bump_width"][0], bed["bump_width"][1],
                                                bed["mound_amp"], bed["mound_width"]))


def one_solve(nmg, prob, tol, reps=1, **over):
    """Status, steps and time per solve (best of reps) of one configuration."""
    import torch
    ctx = nmg.Context.from_problem(prob, **over)
    z = torch.from_numpy(prob.z).cuda()
    ts, st = [], None
    for _ in range(reps):
        U = torch.from_numpy(prob.U0).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.newton_mg_solve(z, U, tol)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ctx.close()
    return dict(status=st["status"], newton_steps=st["newton_steps"],
                init_sweeps=st["init_sweeps"], init_level_sweeps=st["init_level_sweeps"],
                final_res_l1=st["res_l1"], s_per_solve=min(ts),
                solves_per_s=(1.0 / min(ts)) if st["status"] == "OK" else None)


def batched(args):
    """Batched solves of uneven independent problems: `args.batch` steady
    channels with sizes from {128, 256, 384, 512}^2, their own beds and
    inflow discharges U[0.5, 2], FP32 inner W-cycle, FP64 outer, one batch
    solve (after an untimed one) with autotuned tiles."""
    import collections
    import torch
    from paper_1608_06721_amd import nmg
    from paper_1608_06721_amd import workloads as W
    probs = W.batch_channels(args.batch, n_levels=args.batch_levels, gamma=2, inner_fp32=1,
                             max_newton=args.batch_max_newton)
    b = nmg.Batch(probs)
    tiles = b.autotune(reps=5)
    zs = [torch.from_numpy(p.z).cuda() for p in probs]
    U0s = [torch.from_numpy(p.U0).cuda() for p in probs]
    b.newton_mg_solve(zs, [u.clone() for u in U0s], args.tol)
    Us = [u.clone() for u in U0s]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = b.newton_mg_solve(zs, Us, args.tol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    b.close()
    counts = collections.Counter(r["status"] for r in res)
    steps = [r["newton_steps"] for r in res]
    print("[bench] batched: %d instances in %.3f s, %s" % (len(probs), dt, dict(counts)),
          file=sys.stderr, flush=True)
    n_ok = counts.get("OK", 0)
    return {
        # only instances that reached the tolerance count as steady solves
        "value": n_ok / dt, "unit": "solves/s", "instances": len(probs), "converged": n_ok,
        "cells": int(sum(p.nx * p.ny for p in probs)), "ms_per_batch": 1e3 * dt,
        "statuses": dict(counts), "newton_steps_mean": float(sum(steps)) / len(steps),
        "newton_steps_max": max(steps), "max_newton": args.batch_max_newton,
        "n_levels": args.batch_levels, "cycle": "W(2,2), nu_coarse=10, n_mg=3",
        "dtype": "f32 inner / f64 outer", "tiles": tiles,
        "workload": "batch of %d channels, sizes {128,256,384,512}^2, q U[0.5,2] (seed %d), "
                    "bed %s" % (len(probs), W.BATCH_SEED, describe_bed(W.ONE_ISLAND_BED)),
    }


def adjoint_gradients(args):
    """Bed gradients of a gauge misfit on a batch of topographies (512^2
    channels): the objective is the sum over 64 gauges of (h + z - target)^2
    with targets from the steady state over a perturbed bed (one untimed
    batched solve).  Timed: one batched FP64 W-cycle Newton solve of every
    topography, then for each converged one the objective, its adjoint
    multigrid solve (GMRES(30)-accelerated cycles to 1e-12 relative) and the
    bed vector-Jacobian product, the topographies' adjoint solves running
    concurrently on their own contexts and streams.  One untimed round
    first (each context's first adjoint solve allocates its transposed matrix
    and Krylov vectors).  Only converged topographies count."""
    import torch
    from paper_1608_06721_amd import adjoint, nmg
    from paper_1608_06721_amd import workloads as W
    n = args.adjoint_size
    levels = int(math.log2(n)) - 4
    cases = W.gauge_cases(args.adjoint, size=n, n_levels=levels, gamma=2,
                          max_newton=args.max_newton)
    probs = [c.prob for c in cases]
    # targets: steady states over the perturbed beds (one batched solve)
    tb = nmg.Batch(probs)
    Ut = [torch.from_numpy(p.U0).cuda() for p in probs]
    zt = [torch.from_numpy(c.z_true).cuda() for c in cases]
    tres = tb.newton_mg_solve(zt, Ut, args.tol)
    tb.close()
    gauges = [torch.from_numpy(c.gauges).cuda() for c in cases]
    targets = [(Ut[k][0] + zt[k]).reshape(-1)[gauges[k]] for k in range(len(cases))]
    keep = [k for k in range(len(cases)) if tres[k]["status"] == "OK"]
    skipped = ["%s (target solve %s)" % (probs[k].name, tres[k]["status"])
               for k in range(len(cases)) if k not in keep]

    def objective(q, U, z):
        k = keep[q]
        return adjoint.gauge_misfit(U, z, gauges[k], targets[k])

    bg = adjoint.BatchGradients([probs[k] for k in keep], tol=args.tol, adj_tol=1e-12)
    zs = [torch.from_numpy(probs[k].z).cuda() for k in keep]
    U0s = [torch.from_numpy(probs[k].U0).cuda() for k in keep]
    bg(zs, U0s, objective)                         # untimed: first adjoint solves allocate
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    statuses, _, grads, cycles = bg(zs, U0s, objective)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    secs = dict(bg.last_seconds)
    steps = list(bg.newton_steps)
    bg.close()
    ng = sum(g is not None for g in grads)
    skipped += ["%s (steady solve %s)" % (probs[keep[q]].name, statuses[q])
                for q in range(len(keep)) if grads[q] is None]
    print("[bench] adjoint: %d gradients in %.3f s (batched forward %.3f s, concurrent "
          "adjoints %.3f s), %d skipped" % (ng, dt, secs["forward"], secs["adjoint"],
                                            len(skipped)), file=sys.stderr, flush=True)
    return {
        "value": ng / dt if ng else None, "unit": "gradients/s", "topographies": len(cases),
        "gradients": ng, "skipped": skipped, "grid": "%dx%d" % (n, n),
        "ms_per_batch": 1e3 * dt, "ms_forward_batch": 1e3 * secs["forward"],
        "ms_adjoint_concurrent": 1e3 * secs["adjoint"],
        "newton_steps_mean": float(sum(steps)) / max(len(steps), 1),
        "adjoint_cycles_mean": float(sum(c for c in cycles if c)) / max(ng, 1),
        "n_levels": levels, "dtype": "f64", "gauges": 64, "adjoint_rel_tol": 1e-12,
        "workload": "gauge misfit on %d channels %dx%d (seeds %d+b), bed %s; forward solves "
                    "batched, adjoint solves concurrent" % (len(cases), n, n, W.ADJOINT_SEED,
                                                            describe_bed(W.ONE_ISLAND_BED)),
    }


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on the host cores, on a bounded sample.

def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


def level_problem(prob, l):
    """The Step 1 mesh of level l (same domain, (nx, ny) >> l) with the bed
    and initial state averaged over the children level by level, as Step 1
    forms them (input preparation for timing only)."""
    from paper_1608_06721_amd import workloads as W
    z, U = prob.z, prob.U0
    for _ in range(l):
        z = 0.25 * (((z[0::2, 0::2] + z[0::2, 1::2]) + z[1::2, 0::2]) + z[1::2, 1::2])
        U = 0.25 * (((U[:, 0::2, 0::2] + U[:, 0::2, 1::2]) + U[:, 1::2, 0::2]) + U[:, 1::2, 1::2])
    return W.Problem("%s_l%d" % (prob.name, l), prob.dim, prob.nx >> l, prob.ny >> l, prob.x0,
                     prob.x1, prob.y0, prob.y1, prob.bc, dict(prob.params), np.ascontiguousarray(z),
                     np.ascontiguousarray(U))


def oracle_leg(prob, threads, order, level_sweeps, n_newton, budget_s):
    """Times of the oracle (`threads` threads, `order`) for one Newton step at
    the finest level and for one Step 1 BLU-SGS sweep with its residual test
    on each coarse level, and the solve time they project to with the GPU
    solve's counts (the red-black iterates are the GPU's bit for bit, so the
    counts are the oracle's own)."""
    import oracle
    L = oracle.lib()
    L.orc_set_threads(int(threads))
    p = dict(prob.params, order=order)
    t_start = time.perf_counter()
    try:
        t0 = time.perf_counter()
        oracle.newton_solve(prob, tol=0.0, params=dict(p, max_newton=1, eps_p=0.0))
        t_newton = time.perf_counter() - t0
        t_level = {}
        for l, cnt in enumerate(level_sweeps):
            if l == 0 or cnt == 0:
                continue
            if time.perf_counter() - t_start > budget_s:
                break
            pl = level_problem(prob, l)
            reps = max(1, min(20, int(2e5 / (pl.nx * pl.ny))))
            U = pl.U0.copy()
            t0 = time.perf_counter()
            for _ in range(reps):
                oracle.residual(pl, U, p)
                U = oracle.blu_sweep(pl, U, p)
            t_level[l] = (time.perf_counter() - t0) / reps
    finally:
        L.orc_set_threads(1)
    complete = all(l in t_level for l, c in enumerate(level_sweeps) if l > 0 and c > 0)
    step1 = sum(level_sweeps[l] * t for l, t in t_level.items())
    solve = step1 + n_newton * t_newton if complete else None
    return dict(threads=int(threads), order="lexicographic" if order else "red-black",
                s_per_newton_step=t_newton,
                s_per_step1_sweep_by_level={str(l): t for l, t in sorted(t_level.items())},
                projected_s_per_solve=solve,
                projected_solves_per_s=(1.0 / solve) if solve else None,
                sample_s=time.perf_counter() - t_start)


def cpu_baseline(prob, stats, budget_s):
    model, ncpu, avail = host_info()
    threads = max(1, min(16, avail or 1))
    n_newton = stats["newton_steps"]
    lv = stats["init_level_sweeps"]
    print("[bench] CPU oracle: red-black on %d threads" % threads, file=sys.stderr, flush=True)
    rb_mt = oracle_leg(prob, threads, 0, lv, n_newton, budget_s)
    print("[bench] CPU oracle: red-black on 1 thread", file=sys.stderr, flush=True)
    rb_1 = oracle_leg(prob, 1, 0, lv, n_newton, budget_s)
    print("[bench] CPU oracle: lexicographic on 1 thread", file=sys.stderr, flush=True)
    lex_1 = oracle_leg(prob, 1, 1, lv, n_newton, budget_s)
    lex_1["projected_s_per_solve"] = lex_1["projected_solves_per_s"] = None   # other iterates
    return dict(value=rb_mt["projected_solves_per_s"], unit="solves/s", cores=threads,
                kind="oracle",
                sample="one Newton step at %dx%d and one Step 1 BLU-SGS sweep with its residual "
                       "test per coarse level, projected with the GPU solve's %d Newton steps and "
                       "per-level Step 1 sweeps %s" % (prob.nx, prob.ny, n_newton, lv[1:]),
                host_cpu=model, nproc=ncpu, cpus_available=avail,
                legs={"redblack_threads": rb_mt, "redblack_1thread": rb_1,
                      "lexicographic_1thread": lex_1},
                paper_context="the paper's timings are serial on an Intel Core i5 at 3.2 GHz "
                              "(Sec. 3); its 2D example at 512x256 took 13804 s with explicit "
                              "time stepping, NMGM's own 2D times are only plotted")


# ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--max-newton", type=int, default=500)
    ap.add_argument("--v3-max-newton", type=int, default=300,
                    help="step cap of the paper's default V-cycle line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline solve (FP64 and FP32 inner)")
    ap.add_argument("--batch", type=int, default=64,
                    help="instances of the batched-solve workload (0: skip it)")
    ap.add_argument("--batch-levels", type=int, default=5)
    ap.add_argument("--batch-max-newton", type=int, default=150)
    ap.add_argument("--adjoint", type=int, default=16,
                    help="topographies of the gauge-misfit gradient workload (0: skip it)")
    ap.add_argument("--adjoint-size", type=int, default=512)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--timing-cap", type=int, default=20000)
    ap.add_argument("--kernel-probe", action="store_true",
                    help="only run finest-level SGS iterations on the assembled system and a "
                         "512 MiB device copy (for hardware-counter runs), then exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: a single solve is not sharded across GPUs; "
              "run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1608_06721_amd import nmg
    from paper_1608_06721_amd import workloads as W

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    prob = W.benchmark_channel(args.size, max_newton=args.max_newton)
    print("[bench] workload %s levels=%d eps_p=%g tol=%g" % (
        prob.name, prob.params["n_levels"], prob.params["eps_p"], args.tol),
        file=sys.stderr, flush=True)
    z = torch.from_numpy(prob.z).cuda()
    U0 = torch.from_numpy(prob.U0).cuda()
    if args.kernel_probe:
        # Counter calibration: a plain copy of a known size, then 4 block SGS
        # iterations (red, black, red per iteration after the first) on the
        # system assembled at the initial state.
        ctx = nmg.Context.from_problem(prob)
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        dst.copy_(src)
        ctx.assemble_residual_jacobian(z, U0)
        dU = torch.zeros_like(U0)
        ctx.sgs(dU, 4)
        torch.cuda.synchronize()
        print("[bench] kernel probe done", file=sys.stderr, flush=True)
        return

    ctx = nmg.Context.from_problem(prob)
    dt, stats, tm, ph, U64 = timed_solves(ctx, z, U0, args.steps, args.warmup, args.tol,
                                          args.timing_cap, "fp64")
    ctx.close()
    converged = all(st["status"] == "OK" for st in stats)
    last = stats[-1]
    n_newton = last["newton_steps"]
    ms_per_step = 1e3 * dt / args.steps
    phases = {k: v / args.steps for k, v in ph.items()}
    roofline = sgs_roofline(tm, SGS_BYTES_2D, measured_traffic())
    roofline["kernel"] = "k_sgs_half<3, MODE_NORMAL> (finest level)"

    out = {
        "metric": METRIC,
        "value": (args.steps / dt) if converged else None,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "channel_%dx%d_two_islands" % (prob.nx, prob.ny),
            "domain": [0.0, 10.0, 0.0, 2.0],
            "bed": describe_bed(W.BENCH_BED),
            "bc": "inflow discharge 1.0 at x=0, outflow depth 1 at x=10, reflective walls",
            "flux": "LLF", "cycle": describe_cycle(prob.params),
            "step1_eps_p": prob.params["eps_p"],
            "tol": args.tol, "newton_steps": n_newton, "converged": converged,
            "step1_sweeps": last["init_sweeps"],
            "step1_sweeps_by_level": last["init_level_sweeps"],
            "final_res_l1": last["res_l1"],
            "ms_per_newton_step": (ms_per_step - phases["step1"] - phases["final"])
            / max(1, n_newton),
            "phase_ms_per_solve": phases,
        },
        "roofline": roofline,
        "step_roofline": step_roofline(prob, ph, args.steps, n_newton),
    }
    # The same solve with the FP32 inner cycle (hierarchy and smoother in
    # FP32, residual, update and stop test in FP64).
    ctx32 = nmg.Context.from_problem(prob, inner_fp32=1)
    dt32, st32, tm32, ph32, U32 = timed_solves(ctx32, z, U0, args.steps, args.warmup, args.tol,
                                               args.timing_cap, "fp32-inner")
    ctx32.close()
    # error of the FP32-inner steady state against the FP64 one (which equals
    # the FP64 oracle's bit for bit): largest cell difference per component
    dU = (U32 - U64).abs().amax(dim=(1, 2)).tolist()
    scale = U64.abs().amax(dim=(1, 2)).tolist()
    ok32 = all(st["status"] == "OK" for st in st32)
    prob32 = prob.with_params(inner_fp32=1)
    out["fp32_inner"] = {
        "value": (args.steps / dt32) if ok32 else None, "unit": "solves/s",
        "ms_per_step": 1e3 * dt32 / args.steps, "converged": ok32,
        "newton_steps": st32[-1]["newton_steps"], "step1_sweeps": st32[-1]["init_sweeps"],
        "final_res_l1": st32[-1]["res_l1"],
        "max_abs_diff_vs_fp64": {"h": dU[0], "hu": dU[1], "hv": dU[2]},
        "max_abs_fp64": {"h": scale[0], "hu": scale[1], "hv": scale[2]},
        "phase_ms_per_solve": {k: v / args.steps for k, v in ph32.items()},
        "roofline": sgs_roofline(tm32, SGS_BYTES_2D_FP32),
        "step_roofline": step_roofline(prob32, ph32, args.steps, st32[-1]["newton_steps"]),
    }
    if not args.no_extras:
        ex = {}
        # The paper's default multigrid (V(2,2), N_L = 3, Sec. 3) on the same
        # solve, within a step cap.
        pv = W.benchmark_channel(args.size, n_levels=3, gamma=1, max_newton=args.v3_max_newton)
        ex["paper_default_v3"] = dict(one_solve(nmg, pv, args.tol), cycle=describe_cycle(pv.params),
                                      max_newton=args.v3_max_newton)
        print("[bench] V N_L=3: %s" % ex["paper_default_v3"], file=sys.stderr, flush=True)
        # The bed measured before: one emergent island, no Step 1.
        pb = W.benchmark_channel(args.size, bed=W.ONE_ISLAND_BED, eps_p=0.0, n_levels=6,
                                 max_newton=args.max_newton)
        ex["one_island_bed"] = dict(one_solve(nmg, pb, args.tol, reps=3),
                                    bed=describe_bed(W.ONE_ISLAND_BED), step1=False,
                                    cycle=describe_cycle(pb.params))
        print("[bench] one-island bed: %s" % ex["one_island_bed"], file=sys.stderr, flush=True)
        # The paper's 2D wet/dry example (Example 3.7) on its finest mesh.
        ph_ = W.dry_hill(512, 256, n_levels=5, gamma=2, eps_p=0.2, max_newton=args.max_newton)
        ex["dry_hill_512x256"] = dict(one_solve(nmg, ph_, args.tol, reps=3),
                                      cycle=describe_cycle(ph_.params), step1_eps_p=0.2,
                                      example="Example 3.7, dry hill in a channel, LLF")
        print("[bench] dry hill: %s" % ex["dry_hill_512x256"], file=sys.stderr, flush=True)
        out["extras"] = ex
        if args.batch > 0:
            out["batched"] = batched(args)
        if args.adjoint > 0:
            out["adjoint"] = adjoint_gradients(args)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob, last, args.cpu_budget)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
