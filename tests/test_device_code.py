"""Properties of the built gfx950 device code (CPU only: the code object is
taken out of libnmg.so and read with ROCm's LLVM tools).

* No kernel uses generic (flat) loads or stores.  The coarse-cycle kernel and
  the batched kernels take their arrays from tables in device memory; a
  generic access there would also be counted by the LDS wait counter (so
  waits for LDS data would wait for global loads too) and would cap the
  loads a wave keeps in flight.
* No kernel uses scratch memory or spills vector registers.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1608_06721_amd", "libnmg.so")
LLVM = "/opt/rocm/llvm/bin"
TOOLS = ("llvm-objcopy", "clang-offload-bundler", "llvm-objdump", "llvm-readelf")


def tool(name):
    p = os.path.join(LLVM, name)
    return p if os.path.exists(p) else shutil.which(name)


@pytest.fixture(scope="module")
def code_object(tmp_path_factory):
    if not os.path.exists(LIB):
        pytest.skip("libnmg.so is not built")
    if not all(tool(t) for t in TOOLS):
        pytest.skip("ROCm LLVM tools not found")
    d = tmp_path_factory.mktemp("devcode")
    fat = str(d / "fat.bin")
    co = str(d / "dev.co")
    subprocess.run([tool("llvm-objcopy"), "--dump-section=.hip_fatbin=" + fat, LIB, str(d / "x.so")],
                   check=True)
    subprocess.run([tool("clang-offload-bundler"), "--unbundle", "--type=o",
                    "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", "--input=" + fat,
                    "--output=" + co], check=True)
    return co


def test_code_object_holds_the_kernels(code_object):
    syms = subprocess.run([tool("llvm-objdump"), "-t", code_object], check=True,
                          capture_output=True, text=True).stdout
    for k in ("k_coarse_cycle", "k_sgs_half", "k_sgs_pair", "kb_sgs_half", "k_assemble"):
        assert k in syms, k


def test_no_generic_memory_instructions(code_object):
    asm = subprocess.run([tool("llvm-objdump"), "-d", code_object], check=True,
                         capture_output=True, text=True).stdout
    assert "global_load" in asm
    flat = [l.strip() for l in asm.splitlines() if re.search(r"\bflat_(load|store|atomic)", l)]
    assert not flat, "%d generic memory instructions, e.g. %s" % (len(flat), flat[:3])


def test_no_scratch_or_vector_spills(code_object):
    notes = subprocess.run([tool("llvm-readelf"), "--notes", code_object], check=True,
                           capture_output=True, text=True).stdout
    names = re.findall(r"\.symbol:\s+(\S+)", notes)
    scratch = [int(v) for v in re.findall(r"\.private_segment_fixed_size:\s+(\d+)", notes)]
    spills = [int(v) for v in re.findall(r"\.vgpr_spill_count:\s+(\d+)", notes)]
    assert len(names) == len(scratch) == len(spills) > 100
    assert max(scratch) == 0 and max(spills) == 0, [
        n for n, a, b in zip(names, scratch, spills) if a or b][:5]
