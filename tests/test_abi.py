"""CPU-side checks of the C ABI: the gfx950 library builds, loads, and
exports every entry point include/nmg.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest
import torch

from paper_1608_06721_amd import build, nmg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "nmg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nmg_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_api():
    names = declared_functions()
    for required in ("nmg_newton_mg_solve", "nmg_mg_vcycle", "nmg_assemble_residual_jacobian"):
        assert required in names
    assert set(names) == set(nmg.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(build.LIB):
        build.build()
    lib = ctypes.CDLL(build.LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_struct_layouts_match_header():
    """ctypes mirrors of the ABI structs have the sizes the C compiler gives."""
    import subprocess
    import tempfile
    prog = r'''
#include <stdio.h>
#include "nmg.h"
int main(void) { printf("%zu %zu %zu %zu %zu\n", sizeof(nmg_grid), sizeof(nmg_side),
  sizeof(nmg_bc), sizeof(nmg_params), sizeof(nmg_stats)); return 0; }
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(prog)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        sizes = list(map(int, subprocess.run([exe], capture_output=True, text=True,
                                             check=True).stdout.split()))
    assert sizes == [ctypes.sizeof(nmg.nmg_grid), ctypes.sizeof(nmg.nmg_side),
                     ctypes.sizeof(nmg.nmg_bc), ctypes.sizeof(nmg.nmg_params),
                     ctypes.sizeof(nmg.nmg_stats)]



class _StubLib:
    """Stands in for libnmg.so: records which entry points were reached."""

    def __init__(self):
        self.called = []

    def __getattr__(self, name):
        def call(*args):
            self.called.append(name)
            return 0
        return call


@pytest.fixture
def stub_lib(monkeypatch):
    """The binding with a recording stub library and CPU tensors accepted as
    device tensors, so that its argument checks run without a GPU."""
    stub = _StubLib()
    monkeypatch.setattr(nmg, "lib", lambda: stub)
    monkeypatch.setattr(nmg, "_on_device", lambda t: True)
    return stub


def _unopened_context(dim, nx, ny, n_levels):
    """A Context object with the attributes of a (dim, nx, ny) grid and no
    library handle."""
    ctx = nmg.Context.__new__(nmg.Context)
    ctx.dim, ctx.nx, ctx.ny = dim, nx, ny
    ctx.nc = 2 if dim == 1 else 3
    ctx.nb = 3 if dim == 1 else 5
    ctx.n_levels = n_levels
    ctx._h = None
    return ctx


def test_binding_refuses_mis_sized_tensors(stub_lib):
    """Every Context entry point checks each tensor's shape against the grid
    before the library sees its address (the kernels trust the sizes)."""
    ctx = _unopened_context(2, 16, 8, 2)
    f = torch.float64
    z, U = torch.zeros(8, 16, dtype=f), torch.zeros(3, 8, 16, dtype=f)
    bad_U, bad_z = torch.zeros(3, 8, 8, dtype=f), torch.zeros(16, 8, dtype=f)
    calls = [
        lambda: ctx.residual(bad_z, U),
        lambda: ctx.residual(z, bad_U),
        lambda: ctx.residual(z, U, R_out=torch.zeros(2, 8, 16, dtype=f)),
        lambda: ctx.assemble_residual_jacobian(z, bad_U),
        lambda: ctx.mg_vcycle(bad_U),
        lambda: ctx.sgs(U, 1, level=1),                   # level 1 is 8x4
        lambda: ctx.sgs(torch.zeros(3, 2, 4, dtype=f), 1, level=3),   # beyond n_levels
        lambda: ctx.blu_sweep(bad_z, U),
        lambda: ctx.newton_mg_solve(z, bad_U, 1e-10),
        lambda: ctx.load_system(torch.zeros(5, 3, 3, 8, 8, dtype=f), U),
        lambda: ctx.get_system(level=-1),
        lambda: ctx.adjoint_solve(z, U, bad_U, lam=U),
        lambda: ctx.bed_vjp(z, U, U, out=bad_z),
    ]
    for call in calls:
        with pytest.raises(ValueError):
            call()
    assert stub_lib.called == []
    # the same calls with the grid's shapes reach the library
    ctx.residual(z, U, R_out=U.clone())
    ctx.sgs(torch.zeros(3, 4, 8, dtype=f), 1, level=1)
    ctx.bed_vjp(z, U, U, out=z.clone())
    assert stub_lib.called == ["nmg_residual", "nmg_sgs", "nmg_bed_vjp"]


def test_binding_refuses_host_tensors():
    ctx = _unopened_context(2, 16, 8, 2)
    with pytest.raises(TypeError):
        ctx.residual(torch.zeros(8, 16, dtype=torch.float64),
                     torch.zeros(3, 8, 16, dtype=torch.float64))


def test_batch_binding_refuses_mis_sized_tensors(stub_lib):
    b = nmg.Batch.__new__(nmg.Batch)
    b.n = 2
    b.shapes = [((3, 8, 16), (8, 16)), ((3, 16, 16), (16, 16))]
    b._h = None
    f = torch.float64
    zs = [torch.zeros(8, 16, dtype=f), torch.zeros(16, 16, dtype=f)]
    Us = [torch.zeros(3, 8, 16, dtype=f), torch.zeros(3, 16, 16, dtype=f)]
    with pytest.raises(ValueError):
        b.newton_mg_solve(zs, Us[::-1], 1e-10)        # two instances' states swapped
    with pytest.raises(ValueError):
        b.newton_mg_solve(zs[:1], Us, 1e-10)
    assert stub_lib.called == []
