"""GPU parity of batched solves: every instance of a batch (uneven grid
sizes, its own bed and inflow discharge, one parameter set) against the
oracle's solve of that instance alone and against a single-problem GPU
solve, bit for bit, with its own status, step count and residual history.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1608_06721_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-batch]", *a, flush=True)
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


def run_batch(nmg, probs, tol, tune=False):
    b = nmg.Batch(probs)
    if tune:
        tiles = b.autotune(reps=2)
        say("  tiles", tiles)
        assert all(t in (64, 128, 256, 512) for t in tiles)
    zs = [dev(p.z) for p in probs]
    Us = [dev(p.U0) for p in probs]
    res = b.newton_mg_solve(zs, Us, tol, hist_cap=1000)
    b.close()
    return [host(u) for u in Us], res


def check_vs_single(nmg, probs, Ub, rb, tol):
    for p, U, r in zip(probs, Ub, rb):
        ctx = nmg.Context.from_problem(p)
        Us = dev(p.U0)
        st = ctx.newton_mg_solve(dev(p.z), Us, tol)
        ctx.close()
        assert (r["status"], r["newton_steps"], r["n_pinned"]) == \
            (st["status"], st["newton_steps"], st["n_pinned"]), p.name
        assert r["res_l1"] == st["res_l1"] or (np.isnan(r["res_l1"]) and np.isnan(st["res_l1"]))
        np.testing.assert_array_equal(r["res_hist"], st["res_hist"], err_msg=p.name)
        same(U, host(Us), p.name + ": U, batch vs single")


def check_vs_oracle(probs, Ub, rb, tol):
    for p, U, r in zip(probs, Ub, rb):
        Uo, so = oracle.newton_solve(p, tol=tol)
        say("  ", p.name, r["status"], r["newton_steps"], "oracle", so["status"], so["newton_steps"])
        assert (r["status"], r["newton_steps"], r["n_pinned"]) == \
            (so["status"], so["newton_steps"], so["n_pinned"]), p.name
        same(U, Uo, p.name + ": U, batch vs oracle")
        np.testing.assert_allclose(r["res_hist"], so["res_hist"], rtol=1e-12, atol=1e-300)


CASES = {
    # uneven sizes, V-cycle, the coarse kernel on the 8x8..24x24 levels
    "mixed_v": (lambda: W.batch_channels(5, sizes=(32, 64, 96), seed=11, n_levels=2,
                                         max_newton=60), 1e-10, "1024"),
    # W-cycle with the FP32 inner cycle
    "w_fp32": (lambda: W.batch_channels(4, sizes=(32, 64), seed=12, n_levels=3, gamma=2,
                                        inner_fp32=1, max_newton=60), 1e-10, "1024"),
    # every level launched on its own (no coarse kernel), half sweeps fused in pairs
    "launched": (lambda: W.batch_channels(3, sizes=(32, 64), seed=13, n_levels=3, gamma=2,
                                          max_newton=40), 1e-10, "0"),
    # the same with every half sweep launched on its own
    "launched_unfused": (lambda: W.batch_channels(3, sizes=(32, 64), seed=13, n_levels=3, gamma=2,
                                                  max_newton=40), 1e-10, "0", "1"),
    # 1D: two bed families, uneven lengths, the coarse kernel on the 8..25-cell levels
    "one_d": (lambda: [W.bump_1d(64, n_levels=3, max_newton=80),
                       W.smooth_1d(96, n_levels=3, max_newton=80),
                       W.bump_1d(128, n_levels=3, max_newton=80),
                       W.smooth_1d(200, n_levels=3, max_newton=80)], 1e-10, "1024"),
    # a step limit that stops some instances before others converge
    "step_limit": (lambda: W.batch_channels(4, sizes=(32, 64), seed=14, n_levels=3,
                                            max_newton=9), 1e-10, "1024"),
    # the half sweeps on a persistent grid (one block per compute unit) looping
    # over the work list, every level launched with one half sweep per launch
    "persistent": (lambda: W.batch_channels(4, sizes=(32, 64, 96), seed=15, n_levels=3,
                                            gamma=2, max_newton=40), 1e-10, "0", "1", "1"),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_batch_matches_oracle_and_single(nmg, case, monkeypatch):
    mk, tol, cc = CASES[case][:3]
    monkeypatch.setenv("NMG_COARSE_CELLS", cc)
    monkeypatch.setenv("NMG_FUSE", CASES[case][3] if len(CASES[case]) > 3 else "3")
    monkeypatch.setenv("NMG_BATCH_PERSISTENT", CASES[case][4] if len(CASES[case]) > 4 else "0")
    probs = mk()
    say(case, [p.name for p in probs])
    Ub, rb = run_batch(nmg, probs, tol)
    check_vs_oracle(probs, Ub, rb, tol)
    check_vs_single(nmg, probs, Ub, rb, tol)


def test_batch_autotuned_tiles_change_nothing(nmg):
    probs = W.batch_channels(6, sizes=(64, 128, 192), seed=15, n_levels=3, gamma=2,
                             max_newton=80)
    say("autotune", [p.name for p in probs])
    Ua, ra = run_batch(nmg, probs, 1e-10, tune=True)
    check_vs_single(nmg, probs, Ua, ra, 1e-10)


def test_batch_of_one_is_the_single_solve(nmg):
    p = W.channel(64, 32, n_levels=3, gamma=2)
    Ub, rb = run_batch(nmg, [p], 1e-10)
    check_vs_single(nmg, [p], Ub, rb, 1e-10)


def test_batch_rejects_mixed_dims_and_bad_grids(nmg):
    p2 = W.channel(32, 32, n_levels=2)
    p1 = W.bump_1d(200).with_params(n_levels=2)
    with pytest.raises(nmg.NMGError):
        nmg.Batch([p2, p1], params=p2.params)
    with pytest.raises(nmg.NMGError):
        nmg.Batch([p2, W.channel(48, 32)], params=dict(p2.params, n_levels=5))


def test_batch_nonfinite_instance_leaves_the_others_alone(nmg):
    probs = W.batch_channels(3, sizes=(32, 64), seed=16, n_levels=3, max_newton=40)
    U0 = probs[1].U0.copy()
    U0[0, 3, 5] = np.nan
    probs[1] = W.dataclasses.replace(probs[1], U0=U0)
    say("nonfinite", [p.name for p in probs])
    Ub, rb = run_batch(nmg, probs, 1e-10)
    assert rb[1]["status"] == "ENONFINITE" and rb[1]["newton_steps"] == 0
    check_vs_oracle(probs, Ub, rb, 1e-10)
    check_vs_single(nmg, probs, Ub, rb, 1e-10)


def test_full_size_batch_sampled(nmg):
    """The 64-instance workload of the benchmark (sizes up to 512^2, FP32
    inner W-cycle) in its launch configuration (autotuned tiles): sampled
    instances equal their single solves bit for bit, and the smallest one
    also the oracle's."""
    probs = W.batch_channels(64, n_levels=5, gamma=2, inner_fp32=1, max_newton=150)
    b = nmg.Batch(probs)
    say("full batch tiles", b.autotune(reps=2))
    zs = [dev(p.z) for p in probs]
    Us = [dev(p.U0) for p in probs]
    res = b.newton_mg_solve(zs, Us, 1e-10, hist_cap=200)
    b.close()
    Ub = [host(u) for u in Us]
    cells = [p.nx * p.ny for p in probs]
    small = int(np.argmin(cells))
    large = int(np.argmax(cells))
    odd = [k for k, r in enumerate(res) if r["status"] != "OK"][:1]
    sample = sorted({small, large, *odd})
    say("sample", [(probs[k].name, res[k]["status"], res[k]["newton_steps"]) for k in sample])
    check_vs_single(nmg, [probs[k] for k in sample], [Ub[k] for k in sample],
                    [res[k] for k in sample], 1e-10)
    check_vs_oracle([probs[small]], [Ub[small]], [res[small]], 1e-10)
