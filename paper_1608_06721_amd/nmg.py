"""Thin Python binding of libnmg.so (include/nmg.h) over torch device tensors.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Tensors must be torch.float64, contiguous, on the GPU, in the
layouts of include/nmg.h (cell vectors [nc][ny][nx], bed [ny][nx], blocks
[nb][nc][nc][ny][nx]).  There is no CPU fallback: if the library cannot be
loaded, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import torch

from . import build as _build

NMG_OK, NMG_NOT_CONVERGED = 0, 1
STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP",
          -4: "ENONFINITE", -5: "EDIVERGED"}


class nmg_grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double)]


class nmg_side(C.Structure):
    _fields_ = [("kind", C.c_int), ("h", C.c_double), ("qn", C.c_double), ("ut", C.c_double)]


class nmg_bc(C.Structure):
    _fields_ = [("side", nmg_side * 4)]


class nmg_params(C.Structure):
    _fields_ = [("flux", C.c_int), ("g", C.c_double), ("alpha", C.c_double),
                ("fd_eps", C.c_double), ("tau", C.c_double), ("h_eps", C.c_double),
                ("eps_r", C.c_double), ("n_levels", C.c_int), ("nu1", C.c_int),
                ("nu2", C.c_int), ("nu_coarse", C.c_int), ("n_mg", C.c_int),
                ("blu_sweeps", C.c_int), ("max_newton", C.c_int), ("dry_pin", C.c_int),
                ("pos_theta", C.c_double), ("inner_fp32", C.c_int), ("gamma", C.c_int),
                ("eps_p", C.c_double), ("init_max_sweeps", C.c_int)]


class nmg_stats(C.Structure):
    _fields_ = [("newton_steps", C.c_int), ("status", C.c_int), ("n_pinned", C.c_int),
                ("res_l1", C.c_double), ("res_hist", C.POINTER(C.c_double)),
                ("hist_cap", C.c_int), ("init_sweeps", C.c_int),
                ("init_level_sweeps", C.c_int * 16)]


PHASES = ["step1", "blu", "assembly", "galerkin", "norm", "cycles", "update", "final"]


_lib = None
EXPORTS = ["nmg_create", "nmg_destroy", "nmg_last_error", "nmg_residual",
           "nmg_assemble_residual_jacobian", "nmg_mg_vcycle", "nmg_sgs", "nmg_blu_sweep",
           "nmg_newton_mg_solve", "nmg_load_system", "nmg_get_system", "nmg_timing_enable",
           "nmg_timing_read", "nmg_timing_phases", "nmg_batch_create", "nmg_batch_destroy", "nmg_batch_last_error",
           "nmg_batch_autotune", "nmg_batch_newton_mg_solve", "nmg_adjoint_solve",
           "nmg_bed_vjp", "nmg_residual_noalloc"]


def library_path() -> str:
    return _build.LIB


def lib():
    """Load libnmg.so (building it first only if it does not exist)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        vp = C.c_void_p
        L.nmg_create.argtypes = [C.POINTER(nmg_grid), C.POINTER(nmg_bc), C.POINTER(nmg_params),
                                 vp, C.POINTER(vp)]
        L.nmg_destroy.argtypes = [vp]
        L.nmg_destroy.restype = None
        L.nmg_last_error.argtypes = [vp]
        L.nmg_last_error.restype = C.c_char_p
        L.nmg_residual.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_double)]
        L.nmg_assemble_residual_jacobian.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_double)]
        L.nmg_mg_vcycle.argtypes = [vp, vp, C.c_int]
        L.nmg_sgs.argtypes = [vp, C.c_int, vp, C.c_int]
        L.nmg_blu_sweep.argtypes = [vp, vp, vp]
        L.nmg_newton_mg_solve.argtypes = [vp, vp, vp, C.c_double, C.POINTER(nmg_stats)]
        L.nmg_load_system.argtypes = [vp, vp, vp]
        L.nmg_get_system.argtypes = [vp, C.c_int, vp, vp]
        L.nmg_timing_enable.argtypes = [vp, C.c_int, C.c_int]
        L.nmg_timing_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int),
                                      C.POINTER(C.c_longlong)]
        L.nmg_timing_phases.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.nmg_adjoint_solve.argtypes = [vp, vp, vp, vp, vp, C.c_double, C.c_int, C.c_int,
                                        C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.nmg_bed_vjp.argtypes = [vp, vp, vp, vp, vp]
        L.nmg_residual_noalloc.argtypes = [C.POINTER(nmg_grid), C.POINTER(nmg_bc),
                                           C.POINTER(nmg_params), vp, vp, vp, vp, vp]
        L.nmg_batch_create.argtypes = [C.c_int, C.POINTER(nmg_grid), C.POINTER(nmg_bc),
                                       C.POINTER(nmg_params), vp, C.POINTER(vp)]
        L.nmg_batch_destroy.argtypes = [vp]
        L.nmg_batch_destroy.restype = None
        L.nmg_batch_last_error.argtypes = [vp]
        L.nmg_batch_last_error.restype = C.c_char_p
        L.nmg_batch_autotune.argtypes = [vp, C.c_int, C.POINTER(C.c_int)]
        L.nmg_batch_newton_mg_solve.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.c_double,
                                                C.POINTER(nmg_stats)]
        _lib = L
    return _lib


def _on_device(t: torch.Tensor) -> bool:
    return t.is_cuda


def _ptr(t: Optional[torch.Tensor], what: str, shape=None):
    """Device address of `t` after checking its dtype, device, contiguity
    and (if given) its shape: the library trusts the sizes it is passed, so a
    tensor of the wrong size must be refused here rather than read or written
    out of bounds on the GPU."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % what)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (what, tuple(t.shape), tuple(shape)))
    if not _on_device(t) or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("%s must be a contiguous float64 CUDA tensor" % what)
    return C.c_void_p(t.data_ptr())


class NMGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


def _grid(dim, nx, ny, x0, x1, y0, y1):
    return nmg_grid(int(dim), int(nx), int(ny), x0, x1, y0, y1)


def _bc(bc):
    b = nmg_bc()
    for k, s in enumerate(bc):
        b.side[k] = nmg_side(int(s[0]), float(s[1]), float(s[2]), float(s[3]))
    return b


def _params(params):
    return nmg_params(int(params["flux"]), params["g"], params["alpha"], params["fd_eps"],
                      params["tau"], params["h_eps"], params["eps_r"], int(params["n_levels"]),
                      int(params["nu1"]), int(params["nu2"]), int(params["nu_coarse"]),
                      int(params["n_mg"]), int(params["blu_sweeps"]),
                      int(params["max_newton"]), int(params["dry_pin"]),
                      float(params["pos_theta"]), int(params.get("inner_fp32", 0)),
                      int(params.get("gamma", 1)), float(params.get("eps_p", 0.0)),
                      int(params.get("init_max_sweeps", 1000)))


class Context:
    """One grid / boundary condition / parameter set (nmg_create)."""

    def __init__(self, dim, nx, ny, x0, x1, y0, y1, bc, params: dict, stream=None):
        self.dim, self.nx, self.ny = int(dim), int(nx), int(ny)
        self.nc = 2 if self.dim == 1 else 3
        self.nb = 3 if self.dim == 1 else 5
        self.n_levels = int(params["n_levels"])
        g = _grid(self.dim, self.nx, self.ny, x0, x1, y0, y1)
        b = _bc(bc)
        p = _params(params)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        rc = lib().nmg_create(C.byref(g), C.byref(b), C.byref(p), C.c_void_p(stream.cuda_stream),
                              C.byref(h))
        if rc != 0:
            raise NMGError(rc, "nmg_create failed")
        self._h = h

    @classmethod
    def from_problem(cls, prob, stream=None, **overrides):
        params = dict(prob.params)
        params.update(overrides)
        return cls(prob.dim, prob.nx, prob.ny, prob.x0, prob.x1, prob.y0, prob.y1, prob.bc,
                   params, stream)

    def close(self):
        if getattr(self, "_h", None):
            lib().nmg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, ok=(0,)):
        if rc not in ok:
            msg = lib().nmg_last_error(self._h)
            raise NMGError(rc, msg.decode() if msg else "")
        return rc

    def level_shape(self, level):
        nx = self.nx >> level
        ny = 1 if self.dim == 1 else self.ny >> level
        return nx, ny

    def _vec(self, level=0):
        nx, ny = self.level_shape(level)
        return (self.nc, ny, nx)

    def _bed(self):
        return (self.ny, self.nx)

    # --- entry points ------------------------------------------------------
    def residual(self, z, U, R_out=None, want_norm=True):
        res = C.c_double(0.0)
        self._check(lib().nmg_residual(self._h, _ptr(z, "z", self._bed()),
                                       _ptr(U, "U", self._vec()),
                                       _ptr(R_out, "R_out", self._vec()),
                                       C.byref(res) if want_norm else None))
        return res.value if want_norm else None

    def assemble_residual_jacobian(self, z, U, R_out=None, want_norm=True):
        res = C.c_double(0.0)
        self._check(lib().nmg_assemble_residual_jacobian(
            self._h, _ptr(z, "z", self._bed()), _ptr(U, "U", self._vec()),
            _ptr(R_out, "R_out", self._vec()),
            C.byref(res) if want_norm else None))
        return res.value if want_norm else None

    def mg_vcycle(self, dU, n_cycles=1):
        self._check(lib().nmg_mg_vcycle(self._h, _ptr(dU, "dU", self._vec()), int(n_cycles)))

    def sgs(self, dU, iters, level=0):
        if not 0 <= int(level) <= self.n_levels:
            raise ValueError("level %d outside 0..%d" % (level, self.n_levels))
        self._check(lib().nmg_sgs(self._h, int(level), _ptr(dU, "dU", self._vec(level)),
                                  int(iters)))

    def blu_sweep(self, z, U):
        self._check(lib().nmg_blu_sweep(self._h, _ptr(z, "z", self._bed()),
                                        _ptr(U, "U", self._vec())))

    def newton_mg_solve(self, z, U, tol, hist_cap=10000):
        hist = (C.c_double * hist_cap)()
        st = nmg_stats(0, 0, 0, 0.0, C.cast(hist, C.POINTER(C.c_double)), hist_cap, 0)
        n_lev = self.n_levels
        rc = lib().nmg_newton_mg_solve(self._h, _ptr(z, "z", self._bed()),
                                       _ptr(U, "U", self._vec()), float(tol), C.byref(st))
        self._check(rc, ok=(0, 1, -4, -5))
        n = st.newton_steps
        nh = min(n + 1 if rc in (0, -4, -5) else n, hist_cap)
        return dict(status=STATUS.get(rc, rc), newton_steps=n, n_pinned=st.n_pinned,
                    res_l1=st.res_l1, res_hist=[hist[k] for k in range(nh)],
                    init_sweeps=st.init_sweeps,
                    init_level_sweeps=[st.init_level_sweeps[l] for l in range(n_lev + 1)])

    def load_system(self, A0, b0):
        nx, ny = self.level_shape(0)
        self._check(lib().nmg_load_system(self._h,
                                          _ptr(A0, "A0", (self.nb, self.nc, self.nc, ny, nx)),
                                          _ptr(b0, "b0", self._vec())))

    def get_system(self, level=0, want_A=True, want_b=True):
        if not 0 <= int(level) <= self.n_levels:
            raise ValueError("level %d outside 0..%d" % (level, self.n_levels))
        nx, ny = self.level_shape(level)
        dev = torch.device("cuda", torch.cuda.current_device())
        A = torch.empty((self.nb, self.nc, self.nc, ny, nx), dtype=torch.float64, device=dev) \
            if want_A else None
        b = torch.empty((self.nc, ny, nx), dtype=torch.float64, device=dev) if want_b else None
        self._check(lib().nmg_get_system(self._h, int(level), _ptr(A, "A"), _ptr(b, "b")))
        return A, b

    def adjoint_solve(self, z, U, g, lam=None, tol=1e-12, max_cycles=200, krylov=0):
        """Solve (dR/dU)^T lam = g at (z, U) by multigrid cycles, GMRES(krylov)
        accelerated if krylov > 0 (nmg_adjoint_solve); returns (lam, cycles,
        relative l1 residual)."""
        if lam is None:
            lam = torch.zeros_like(g)
        cyc, rel = C.c_int(0), C.c_double(0.0)
        v = self._vec()
        self._check(lib().nmg_adjoint_solve(self._h, _ptr(z, "z", self._bed()), _ptr(U, "U", v),
                                            _ptr(g, "g", v), _ptr(lam, "lambda", v),
                                            float(tol), int(max_cycles),
                                            int(krylov), C.byref(cyc), C.byref(rel)))
        return lam, cyc.value, rel.value

    def bed_vjp(self, z, U, lam, out=None):
        """(dR/dz)^T lam at (z, U) as a [ny][nx] tensor (nmg_bed_vjp)."""
        if out is None:
            out = torch.empty_like(z)
        v = self._vec()
        self._check(lib().nmg_bed_vjp(self._h, _ptr(z, "z", self._bed()), _ptr(U, "U", v),
                                      _ptr(lam, "lambda", v), _ptr(out, "out", self._bed())))
        return out

    def timing_enable(self, enable=True, cap=4096):
        self._check(lib().nmg_timing_enable(self._h, int(bool(enable)), int(cap)))

    def timing_phases(self):
        """Stream time per phase of the recorded Newton solves (ms), by name."""
        ms = (C.c_double * len(PHASES))()
        marks = C.c_int(0)
        self._check(lib().nmg_timing_phases(self._h, ms, C.byref(marks)))
        out = {name: ms[k] for k, name in enumerate(PHASES)}
        out["marks"] = marks.value
        return out

    def timing_read(self):
        ms, n, cells = C.c_double(0), C.c_int(0), C.c_longlong(0)
        self._check(lib().nmg_timing_read(self._h, C.byref(ms), C.byref(n), C.byref(cells)))
        return dict(ms=ms.value, launches=n.value, cells=cells.value)


def residual_noalloc(prob, z, U, R_out=None, res_l1=None, stream=None):
    """nmg_residual_noalloc: residuals of U over z for the grid, boundary
    data and physics of `prob` (anything with the attributes of
    workloads.Problem) without a context or any allocation by the library;
    R_out (nullable, [nc][ny][nx]) and res_l1 (nullable, a one-element
    float64 device tensor for sum_i ||R_i||_1) are filled on `stream`
    (default: torch's current stream) without synchronizing."""
    nc = 2 if prob.dim == 1 else 3
    vec, bed = (nc, prob.ny, prob.nx), (prob.ny, prob.nx)
    g = _grid(prob.dim, prob.nx, prob.ny, prob.x0, prob.x1, prob.y0, prob.y1)
    b = _bc(prob.bc)
    p = _params(prob.params)
    if stream is None:
        stream = torch.cuda.current_stream()
    rc = lib().nmg_residual_noalloc(C.byref(g), C.byref(b), C.byref(p),
                                    C.c_void_p(stream.cuda_stream), _ptr(z, "z", bed),
                                    _ptr(U, "U", vec), _ptr(R_out, "R_out", vec),
                                    _ptr(res_l1, "res_l1", (1,)))
    if rc != 0:
        raise NMGError(rc, "nmg_residual_noalloc refused the call (invalid arguments, or more "
                           "than 2^26 cells)" if rc == -1 else "nmg_residual_noalloc failed")


def newton_mg_solve(prob, z, U, tol, stream=None, **overrides):
    """Convenience: create a context for `prob` and solve in place from U."""
    ctx = Context.from_problem(prob, stream, **overrides)
    try:
        return ctx.newton_mg_solve(z, U, tol)
    finally:
        ctx.close()


class Batch:
    """Independent problems solved in lockstep (nmg_batch_create): each
    problem's own grid and boundary data, one parameter set for all."""

    def __init__(self, probs, params: Optional[dict] = None, stream=None, **overrides):
        n = len(probs)
        if n < 1:
            raise ValueError("empty batch")
        params = dict(params if params is not None else probs[0].params)
        params.update(overrides)
        self.n = n
        self.params = params
        nc = 2 if probs[0].dim == 1 else 3
        self.shapes = [((nc, p.ny, p.nx), (p.ny, p.nx)) for p in probs]
        grids = (nmg_grid * n)(*[_grid(p.dim, p.nx, p.ny, p.x0, p.x1, p.y0, p.y1) for p in probs])
        bcs = (nmg_bc * n)(*[_bc(p.bc) for p in probs])
        prm = _params(params)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        rc = lib().nmg_batch_create(n, grids, bcs, C.byref(prm), C.c_void_p(stream.cuda_stream),
                                    C.byref(h))
        if rc != 0:
            raise NMGError(rc, "nmg_batch_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().nmg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, ok=(0,)):
        if rc not in ok:
            msg = lib().nmg_batch_last_error(self._h)
            raise NMGError(rc, msg.decode() if msg else "")
        return rc

    def autotune(self, reps=5):
        """Pick the tile length of the batched half sweep per level; returns
        the chosen lengths (levels 0..n_levels)."""
        nl = int(self.params["n_levels"])
        out = (C.c_int * (nl + 1))()
        self._check(lib().nmg_batch_autotune(self._h, int(reps), out))
        return list(out)

    def newton_mg_solve(self, zs, Us, tol, hist_cap=0):
        """Solve every instance in place from Us[k]; returns one result dict
        per instance (as Context.newton_mg_solve)."""
        if len(zs) != self.n or len(Us) != self.n:
            raise ValueError("need one z and one U per instance")
        zp = (C.c_void_p * self.n)(*[_ptr(z, "z[%d]" % k, self.shapes[k][1])
                                     for k, z in enumerate(zs)])
        up = (C.c_void_p * self.n)(*[_ptr(u, "U[%d]" % k, self.shapes[k][0])
                                     for k, u in enumerate(Us)])
        hists = [(C.c_double * max(hist_cap, 1))() for _ in range(self.n)]
        st = (nmg_stats * self.n)()
        for k in range(self.n):
            st[k] = nmg_stats(0, 0, 0, 0.0,
                              C.cast(hists[k], C.POINTER(C.c_double)) if hist_cap else None,
                              int(hist_cap), 0)
        rc = lib().nmg_batch_newton_mg_solve(self._h, zp, up, float(tol), st)
        self._check(rc, ok=(0, 1))
        out = []
        for k in range(self.n):
            s = st[k]
            n = s.newton_steps
            nh = min(n + 1 if s.status in (0, -4, -5) else n, hist_cap)
            out.append(dict(status=STATUS.get(s.status, s.status), newton_steps=n,
                            n_pinned=s.n_pinned, res_l1=s.res_l1,
                            res_hist=[hists[k][q] for q in range(nh)]))
        return out
