"""ctypes wrapper of the plain FP64 CPU oracle (oracle/nmg_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg import this package.  It shares no code with
the GPU path; problems are passed in as duck-typed objects with the
attributes of ``paper_1608_06721_amd.workloads.Problem`` (dim, nx, ny, x0,
x1, y0, y1, bc, params, z).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

REDBLACK, LEX = 0, 1
STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -4: "ENONFINITE", -5: "EDIVERGED"}


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double)]


class SideBC(C.Structure):
    _fields_ = [("kind", C.c_int), ("h", C.c_double), ("qn", C.c_double), ("ut", C.c_double)]


class Params(C.Structure):
    _fields_ = [("flux", C.c_int), ("g", C.c_double), ("alpha", C.c_double),
                ("fd_eps", C.c_double), ("tau", C.c_double), ("h_eps", C.c_double),
                ("eps_r", C.c_double), ("n_levels", C.c_int), ("nu1", C.c_int),
                ("nu2", C.c_int), ("nu_coarse", C.c_int), ("n_mg", C.c_int),
                ("blu_sweeps", C.c_int), ("max_newton", C.c_int), ("order", C.c_int),
                ("dry_pin", C.c_int), ("pos_theta", C.c_double), ("inner_fp32", C.c_int),
                ("gamma", C.c_int), ("eps_p", C.c_double), ("init_max_sweeps", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("newton_steps", C.c_int), ("status", C.c_int), ("n_pinned", C.c_int),
                ("res_l1", C.c_double), ("res_hist", C.POINTER(C.c_double)),
                ("hist_cap", C.c_int), ("init_sweeps", C.c_int)]


def lib():
    """Load the oracle library, compiling it first if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = C.CDLL(_build.LIB)
        _lib.orc_inflow_celerity.restype = C.c_double
    return _lib


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _grid(prob):
    return Grid(prob.dim, prob.nx, prob.ny, prob.x0, prob.x1, prob.y0, prob.y1)


def _bc(prob):
    arr = (SideBC * 4)()
    for k, s in enumerate(prob.bc):
        arr[k] = SideBC(int(s[0]), float(s[1]), float(s[2]), float(s[3]))
    return arr


def params_struct(p: dict) -> Params:
    return Params(int(p["flux"]), p["g"], p["alpha"], p["fd_eps"], p["tau"], p["h_eps"],
                  p["eps_r"], int(p["n_levels"]), int(p["nu1"]), int(p["nu2"]),
                  int(p["nu_coarse"]), int(p["n_mg"]), int(p["blu_sweeps"]),
                  int(p["max_newton"]), int(p["order"]), int(p["dry_pin"]),
                  float(p["pos_theta"]), int(p.get("inner_fp32", 0)), int(p.get("gamma", 1)),
                  float(p.get("eps_p", 0.0)), int(p.get("init_max_sweeps", 1000)))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc < 0:
        raise RuntimeError("oracle %s failed: %s" % (what, STATUS.get(rc, rc)))
    return rc


# --- unit pieces -------------------------------------------------------------
def num_flux(flux, nc, axis, g, eps_r, hL, uL, vL, hR, uR, vR):
    out = np.zeros(3)
    lib().orc_num_flux(C.c_int(flux), C.c_int(nc), C.c_int(axis), C.c_double(g),
                       C.c_double(eps_r), *[C.c_double(float(v)) for v in (hL, uL, vL, hR, uR, vR)],
                       _dp(out))
    return out[:nc]


def phys_flux(nc, axis, g, h, u, v):
    out = np.zeros(3)
    lib().orc_phys_flux(C.c_int(nc), C.c_int(axis), C.c_double(g), C.c_double(h),
                        C.c_double(u), C.c_double(v), _dp(out))
    return out[:nc]


def ghost(side, f, g, h_eps, h, u, v):
    s = SideBC(int(side[0]), float(side[1]), float(side[2]), float(side[3]))
    out = np.zeros(3)
    lib().orc_ghost(C.byref(s), C.c_int(f), C.c_double(g), C.c_double(h_eps),
                    C.c_double(h), C.c_double(u), C.c_double(v), _dp(out))
    return out


def inflow_celerity(K, gq):
    return lib().orc_inflow_celerity(C.c_double(K), C.c_double(gq))


def solve_block(D, r):
    D = _f64(D)
    r = _f64(r)
    nc = r.shape[0]
    x = np.zeros(nc)
    lib().orc_solve_block(C.c_int(nc), _dp(D), _dp(r), _dp(x))
    return x


# --- discretization -----------------------------------------------------------
def residual(prob, U, params=None):
    p = params_struct(params or prob.params)
    U = _f64(U)
    R = np.zeros_like(U)
    tot = C.c_double(0.0)
    _check(lib().orc_residual(C.byref(_grid(prob)), _bc(prob), C.byref(p), _dp(_f64(prob.z)),
                              _dp(U), _dp(R), C.byref(tot)), "residual")
    return R, tot.value


def isolated(prob, U):
    p = params_struct(prob.params)
    iso = np.zeros((prob.ny, prob.nx), dtype=np.uint8)
    _check(lib().orc_isolated(C.byref(_grid(prob)), _bc(prob), C.byref(p), _dp(_f64(prob.z)),
                              _dp(_f64(U)), iso.ctypes.data_as(C.POINTER(C.c_ubyte))), "isolated")
    return iso.astype(bool)


def assemble(prob, U, params=None):
    """Level-0 system at U: A [nb][nc][nc][ny][nx], b = -R (0 at pinned cells),
    and sum_i ||R_i||_1."""
    p = params_struct(params or prob.params)
    nc, nb = prob.nc, prob.nb
    A = np.zeros((nb, nc, nc, prob.ny, prob.nx))
    b = np.zeros((nc, prob.ny, prob.nx))
    tot = C.c_double(0.0)
    _check(lib().orc_assemble(C.byref(_grid(prob)), _bc(prob), C.byref(p), _dp(_f64(prob.z)),
                              _dp(_f64(U)), _dp(A), _dp(b), C.byref(tot)), "assemble")
    return A, b, tot.value


# --- linear multigrid ----------------------------------------------------------
def _dims(A):
    nb, nc, _, ny, nx = A.shape
    return (1 if nb == 3 else 2), nx, ny, nc, nb


def galerkin(A):
    dim, nx, ny, nc, nb = _dims(A)
    Ac = np.zeros((nb, nc, nc, max(ny // 2, 1) if dim == 2 else 1, nx // 2))
    lib().orc_galerkin(C.c_int(dim), C.c_int(nx), C.c_int(ny), _dp(_f64(A)), _dp(Ac))
    return Ac


def hierarchy(A0, n_levels):
    out = [_f64(A0)]
    for _ in range(n_levels):
        out.append(galerkin(out[-1]))
    return out


def sgs_half(A, b, x, color):
    dim, nx, ny, nc, nb = _dims(A)
    x = _f64(x).copy()
    lib().orc_sgs_half(C.c_int(dim), C.c_int(nx), C.c_int(ny), _dp(_f64(A)), _dp(_f64(b)),
                       _dp(x), C.c_int(color))
    return x


def sgs(A, b, x, iters, order=REDBLACK):
    dim, nx, ny, nc, nb = _dims(A)
    x = _f64(x).copy()
    lib().orc_sgs(C.c_int(dim), C.c_int(nx), C.c_int(ny), _dp(_f64(A)), _dp(_f64(b)), _dp(x),
                  C.c_int(iters), C.c_int(order))
    return x


def lin_residual(A, b, x):
    dim, nx, ny, nc, nb = _dims(A)
    r = np.zeros_like(_f64(b))
    lib().orc_lin_residual(C.c_int(dim), C.c_int(nx), C.c_int(ny), _dp(_f64(A)), _dp(_f64(b)),
                           _dp(_f64(x)), _dp(r))
    return r


def restrict(A, b, x):
    dim, nx, ny, nc, nb = _dims(A)
    bc = np.zeros((nc, ny // 2 if dim == 2 else 1, nx // 2))
    lib().orc_restrict(C.c_int(dim), C.c_int(nx), C.c_int(ny), _dp(_f64(A)), _dp(_f64(b)),
                       _dp(_f64(x)), _dp(bc))
    return bc


def prolong(xc, x):
    nc, ny, nx = x.shape
    dim = 1 if nc == 2 else 2
    x = _f64(x).copy()
    lib().orc_prolong(C.c_int(dim), C.c_int(nx), C.c_int(ny), _dp(_f64(xc)), _dp(x))
    return x


def vcycles(A0, b0, x, params, n_cycles=1):
    dim, nx, ny, nc, nb = _dims(A0)
    x = _f64(x).copy()
    p = params_struct(params)
    _check(lib().orc_vcycles(C.c_int(dim), C.c_int(nx), C.c_int(ny), C.byref(p), _dp(_f64(A0)),
                             _dp(_f64(b0)), _dp(x), C.c_int(n_cycles)), "vcycles")
    return x


# --- nonlinear driver ------------------------------------------------------------
def blu_sweep(prob, U, params=None):
    p = params_struct(params or prob.params)
    U = _f64(U).copy()
    _check(lib().orc_blu_sweep(C.byref(_grid(prob)), _bc(prob), C.byref(p), _dp(_f64(prob.z)),
                               _dp(U)), "blu_sweep")
    return U


def threshold(prob, U, params=None):
    p = params_struct(params or prob.params)
    U = _f64(U).copy()
    lib().orc_threshold(C.byref(_grid(prob)), C.byref(p), _dp(U))
    return U


def newton_solve(prob, U0=None, tol=1e-10, params=None, hist_cap=10000):
    """Newton multigrid solve (Algorithm 1, Steps 2-3) from U0; returns
    (U, stats dict)."""
    p = params_struct(params or prob.params)
    U = _f64(prob.U0 if U0 is None else U0).copy()
    hist = np.zeros(hist_cap)
    st = Stats(0, 0, 0, 0.0, _dp(hist), hist_cap, 0)
    rc = lib().orc_newton_solve(C.byref(_grid(prob)), _bc(prob), C.byref(p), _dp(_f64(prob.z)),
                                _dp(U), C.c_double(tol), C.byref(st))
    n = st.newton_steps
    nh = min(n + 1, hist_cap) if st.status in (0, -4, -5) else min(n, hist_cap)
    return U, dict(status=STATUS.get(rc, rc), newton_steps=n, n_pinned=st.n_pinned,
                   res_l1=st.res_l1, res_hist=hist[:nh].copy(), init_sweeps=st.init_sweeps)


def nested_init(prob, U0=None, params=None):
    """Algorithm 1, Step 1 from U0 (default prob.U0): returns (Newton's initial
    guess, BLU-SGS sweeps per level)."""
    p = params_struct(params or prob.params)
    U = _f64(prob.U0 if U0 is None else U0).copy()
    sw = (C.c_int * 16)()
    _check(lib().orc_nested_init(C.byref(_grid(prob)), _bc(prob), C.byref(p), _dp(_f64(prob.z)),
                                 _dp(U), sw), "nested_init")
    return U, [sw[l] for l in range(int(p.n_levels) + 1)]


# --- sensitivities ---------------------------------------------------------------
def transpose_blocks(A):
    """Exact block transpose of a level matrix (the adjoint system's matrix)."""
    dim, nx, ny, nc, nb = _dims(A)
    At = np.zeros_like(_f64(A))
    lib().orc_transpose_blocks(C.c_int(dim), C.c_int(nx), C.c_int(ny), _dp(_f64(A)), _dp(At))
    return At


def bed_vjp(prob, U, lam, params=None):
    """(dR/dz)^T lam [ny][nx] by forward differences in the bed, rows pinned
    as in the assembly."""
    p = params_struct(params or prob.params)
    out = np.zeros((prob.ny, prob.nx))
    _check(lib().orc_bed_vjp(C.byref(_grid(prob)), _bc(prob), C.byref(p), _dp(_f64(prob.z)),
                             _dp(_f64(U)), _dp(_f64(lam)), _dp(out)), "bed_vjp")
    return out
