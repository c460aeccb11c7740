"""CPU-side checks of the C ABI: the gfx950 library builds, loads, and
exports every entry point include/nmg.h declares (no compute calls here)."""
import ctypes
import os
import re

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
