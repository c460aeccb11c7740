#!/usr/bin/env python3
"""Benchmark of the Newton multigrid steady shallow-water solver on one MI355X.

One step = one steady solve of the 2D channel workload (1024 x 1024 cells,
FP64): from the resting initial state resident in HBM to sum_i ||R_i||_1 <
tol, i.e. every part of the hot path (BLU-SGS pre-smoothing, residual and
FD-Jacobian assembly, Galerkin coarsening, red-black block-SGS V-cycles,
relaxed update) as many Newton steps as the solve needs.

Prints one JSON line with the metric, the roofline of the dominant kernel
(the finest-level block SGS half sweep, timed with hipEvents on the
library's stream) and the CPU oracle timed on a bounded sample.
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


def workload(args):
    from paper_1608_06721_amd import workloads as W
    n = args.size
    levels = args.levels if args.levels is not None else int(math.log2(n)) - 2
    prob = W.channel(n, n, n_levels=levels, max_newton=args.max_newton,
                     bump_width=tuple(args.bump_width), mound_amp=args.mound_amp,
                     gamma=args.gamma)
    return prob


def cpu_baseline(prob, n_steps, budget_s):
    """The oracle (single thread) on a bounded sample of the same solve:
    as many whole Newton steps as fit the budget (at least one), scaled to
    solves/s with the solve's step count."""
    import oracle
    p = dict(prob.params)
    t0 = time.time()
    done = 0
    U = prob.U0.copy()
    while True:
        U, _ = oracle.newton_solve(prob, U0=U, tol=0.0, params=dict(p, max_newton=1))
        done += 1
        if time.time() - t0 > budget_s * 0.5 or done >= max(1, n_steps):
            break
    dt = time.time() - t0
    per_step = dt / done
    return dict(value=1.0 / (per_step * max(1, n_steps)), unit="solves/s", cores=1,
                kind="oracle",
                sample="%d Newton step(s) of the same %dx%d solve in %.1f s on one host core, "
                       "scaled by the solve's %d steps" % (done, prob.nx, prob.ny, dt, n_steps),
                s_per_newton_step=per_step)


def timed_solves(ctx, z, U0, steps, warmup, tol, cap):
    """Warm-up solves, then `steps` timed solves from U0 (inputs resident in
    HBM); returns (seconds, stats, timing of the finest full SGS sweeps, the
    last solve's state)."""
    import torch
    for _ in range(warmup):
        ctx.newton_mg_solve(z, U0.clone(), tol)
    Us = [U0.clone() for _ in range(steps)]
    ctx.timing_enable(True, cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [ctx.newton_mg_solve(z, Us[k], tol) for k in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.timing_enable(False)
    return dt, stats, ctx.timing_read(), Us[-1]


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
        "workload": "batch of %d channels, sizes {128,256,384,512}^2, q U[0.5,2] (seed %d)"
                    % (len(probs), W.BATCH_SEED),
    }


def adjoint_gradients(args):
    """Bed gradients of a gauge misfit: for each of `args.adjoint`
    topographies (512^2 channels), the steady state (FP64 W-cycle Newton
    multigrid), the objective sum over 64 gauges of (h + z - target)^2 with
    targets from the steady state over a perturbed bed (untimed), and its
    gradient through the autograd Function (adjoint multigrid solve to 1e-12
    relative, then the bed vector-Jacobian product).  Timed: forward solve +
    objective + backward, per topography, after one untimed gradient of the
    first topography with a steady state (the first backward pass allocates
    the adjoint's matrix and Krylov buffers and loads its kernels: 0.6 s
    against ~0.06 s for the later ones)."""
    import torch
    from paper_1608_06721_amd import adjoint, nmg
    from paper_1608_06721_amd import workloads as W
    n = args.adjoint_size
    levels = int(math.log2(n)) - 4
    cases = W.gauge_cases(args.adjoint, size=n, n_levels=levels, gamma=2,
                          max_newton=args.max_newton)
    ctx = nmg.Context.from_problem(cases[0].prob)
    times, fwd, adj, steps, skipped = [], [], [], [], []
    warm = True
    for c in cases:
        p = c.prob
        Ut = torch.from_numpy(p.U0).cuda()
        st = ctx.newton_mg_solve(torch.from_numpy(c.z_true).cuda(), Ut, args.tol)
        if st["status"] != "OK":           # no steady state, no target: not a gradient case
            skipped.append("%s (target solve %s)" % (p.name, st["status"]))
            continue
        g = torch.from_numpy(c.gauges).cuda()
        target = (Ut[0] + torch.from_numpy(c.z_true).cuda()).reshape(-1)[g]
        U0 = torch.from_numpy(p.U0).cuda()
        if warm:
            warm = False
            try:
                zw = torch.from_numpy(p.z).cuda().requires_grad_(True)
                adjoint.gauge_misfit(adjoint.steady_state(ctx, zw, U0, tol=args.tol,
                                                          adj_tol=1e-12), zw, g, target).backward()
            except nmg.NMGError:
                warm = True             # no gradient here: warm up on the next topography
        z = torch.from_numpy(p.z).cuda().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            U = adjoint.steady_state(ctx, z, U0, tol=args.tol, adj_tol=1e-12)
        except nmg.NMGError as e:
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            skipped.append("%s (%s)" % (p.name, e))
            continue
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J = adjoint.gauge_misfit(U, z, g, target)
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append(t2 - t0)
        fwd.append(t1 - t0)
        adj.append(t2 - t1)
        steps.append(U.grad_fn.stats["newton_steps"])
    ctx.close()
    tot = sum(times)
    ng = len(fwd)
    print("[bench] adjoint: %d gradients in %.3f s (forward %.3f s), %d skipped"
          % (ng, tot, sum(fwd), len(skipped)), file=sys.stderr, flush=True)
    return {
        "value": ng / tot if ng else None, "unit": "gradients/s", "topographies": len(cases),
        "gradients": ng, "skipped": skipped,
        "grid": "%dx%d" % (n, n), "ms_per_gradient": 1e3 * tot / max(ng, 1),
        "ms_forward_mean": 1e3 * sum(fwd) / max(ng, 1),
        "ms_adjoint_mean": 1e3 * sum(adj) / max(ng, 1),
        "newton_steps_mean": float(sum(steps)) / max(len(steps), 1), "n_levels": levels,
        "dtype": "f64", "gauges": 64, "adjoint_rel_tol": 1e-12,
        "workload": "gauge misfit on %d channels %dx%d (seeds %d+b)" % (len(cases), n, n,
                                                                      W.ADJOINT_SEED),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--size", type=int, default=1024)
    # W-cycle (gamma = 2) on 7 levels (coarsest 16x16): 39 Newton steps on the
    # channel against 216 for the V-cycle on 9 levels, which is 2.2x slower.
    ap.add_argument("--levels", type=int, default=6)
    ap.add_argument("--gamma", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--max-newton", type=int, default=500)
    # Bed of the measured channel: 16 seeded Gaussians (amplitude U[0, 0.3],
    # width U[0.2, 0.8]) and two mounds of amplitude 0.8 (one emerges as a
    # dry island).  With narrower bumps (widths U[0.05, 0.4]) or mounds of
    # amplitude 0.9 and more the method does not converge at 1024^2.
    ap.add_argument("--bump-width", type=float, nargs=2, default=[0.2, 0.8])
    ap.add_argument("--mound-amp", type=float, default=0.8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=64,
                    help="instances of the batched-solve workload (0: skip it)")
    ap.add_argument("--batch-levels", type=int, default=5)
    ap.add_argument("--batch-max-newton", type=int, default=150)
    ap.add_argument("--adjoint", type=int, default=16,
                    help="topographies of the gauge-misfit gradient workload (0: skip it)")
    ap.add_argument("--adjoint-size", type=int, default=512)
    ap.add_argument("--cpu-budget", type=float, default=30.0)
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

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    prob = workload(args)
    print("[bench] workload %s levels=%d tol=%g" % (prob.name, prob.params["n_levels"], args.tol),
          file=sys.stderr, flush=True)
    ctx = nmg.Context.from_problem(prob)
    z = torch.from_numpy(prob.z).cuda()
    U0 = torch.from_numpy(prob.U0).cuda()
    if args.kernel_probe:
        # Counter calibration: a plain copy of a known size, then 4 block SGS
        # iterations (red, black, red per iteration after the first) on the
        # system assembled at the initial state.
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
    Us = [U0.clone() for _ in range(args.steps)]
    torch.cuda.synchronize()

    for w in range(args.warmup):
        U = U0.clone()
        st = ctx.newton_mg_solve(z, U, args.tol)
        print("[bench] warmup %d: %s steps=%d res=%.3e" % (w, st["status"], st["newton_steps"],
                                                          st["res_l1"]),
              file=sys.stderr, flush=True)

    ctx.timing_enable(True, args.timing_cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.steps):
        stats.append(ctx.newton_mg_solve(z, Us[k], args.tol))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.timing_enable(False)
    tm = ctx.timing_read()
    for k, st in enumerate(stats):
        print("[bench] solve %d: %s steps=%d res=%.3e" % (k, st["status"], st["newton_steps"],
                                                         st["res_l1"]),
              file=sys.stderr, flush=True)
    converged = all(st["status"] == "OK" for st in stats)
    n_newton = stats[-1]["newton_steps"]
    ms_per_step = 1e3 * dt / args.steps

    avg_ms = tm["ms"] / max(1, tm["launches"])
    cells_per_launch = tm["cells"] / max(1, tm["launches"])
    bytes_per_launch = cells_per_launch * SGS_BYTES_2D
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if tm["launches"] else None
    traffic = measured_traffic()
    roofline = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=(achieved / HBM_PEAK_GBS) if achieved else None,
                    traffic=(traffic / (avg_ms * 1e-3) / 1e9) if (traffic and achieved) else None,
                    traffic_bytes_per_launch=traffic,
                    kernel="k_sgs_half<3, MODE_NORMAL> (finest level)",
                    avg_launch_us=avg_ms * 1e3, launches=tm["launches"],
                    bytes_per_launch=bytes_per_launch)

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
            "workload": "channel_%dx%d" % (prob.nx, prob.ny),
            "domain": [0.0, 10.0, 0.0, 2.0],
            "bed": "16 seeded Gaussians (amp U[0,0.3], width U[%g,%g]) + 2 mounds of "
                   "amplitude %g, width 0.25 (seed %d)" % (args.bump_width[0], args.bump_width[1],
                                                         args.mound_amp, 160806721),
            "flux": "LLF", "n_levels": prob.params["n_levels"],
            "cycle": "%s(%d,%d), nu_coarse=%d, n_mg=%d" % (
                "V" if prob.params["gamma"] == 1 else "W", prob.params["nu1"], prob.params["nu2"],
                prob.params["nu_coarse"], prob.params["n_mg"]),
            "tol": args.tol, "newton_steps": n_newton, "converged": converged,
            "final_res_l1": stats[-1]["res_l1"],
            "ms_per_newton_step": ms_per_step / max(1, n_newton),
        },
        "roofline": roofline,
    }
    # The same solve with the FP32 inner V-cycle (hierarchy and smoother in
    # FP32, residual, update and stop test in FP64).
    ctx32 = nmg.Context.from_problem(prob, inner_fp32=1)
    dt32, st32, tm32, U32 = timed_solves(ctx32, z, U0, args.steps, args.warmup, args.tol,
                                         args.timing_cap)
    # error of the FP32-inner steady state against the FP64 one (which equals
    # the FP64 oracle's bit for bit): largest cell difference per component
    dU = (U32 - Us[-1]).abs().amax(dim=(1, 2)).tolist()
    scale = Us[-1].abs().amax(dim=(1, 2)).tolist()
    ok32 = all(st["status"] == "OK" for st in st32)
    avg32 = tm32["ms"] / max(1, tm32["launches"])
    bpl32 = tm32["cells"] / max(1, tm32["launches"]) * SGS_BYTES_2D_FP32
    ach32 = bpl32 / (avg32 * 1e-3) / 1e9 if tm32["launches"] else None
    out["fp32_inner"] = {
        "value": (args.steps / dt32) if ok32 else None, "unit": "solves/s",
        "ms_per_step": 1e3 * dt32 / args.steps, "converged": ok32,
        "newton_steps": st32[-1]["newton_steps"], "final_res_l1": st32[-1]["res_l1"],
        "max_abs_diff_vs_fp64": {"h": dU[0], "hu": dU[1], "hv": dU[2]},
        "max_abs_fp64": {"h": scale[0], "hu": scale[1], "hv": scale[2]},
        "roofline": {"bound": "hbm", "achieved": ach32, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (ach32 / HBM_PEAK_GBS) if ach32 else None,
                     "avg_launch_us": avg32 * 1e3, "bytes_per_launch": bpl32},
    }
    print("[bench] fp32-inner: %s steps=%d %.3f s/solve" % (ok32, st32[-1]["newton_steps"],
                                                           dt32 / args.steps),
          file=sys.stderr, flush=True)
    ctx32.close()
    if args.batch > 0:
        out["batched"] = batched(args)
    if args.adjoint > 0:
        out["adjoint"] = adjoint_gradients(args)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob, n_newton, args.cpu_budget)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
