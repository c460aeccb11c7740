"""Build the oracle's shared library (plain C, FP64, no contraction).

Test infrastructure only: the library is the CPU oracle the GPU path is
checked against.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nmg_oracle.c")
LIB = os.path.join(HERE, "libnmg_oracle.so")

CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-fopenmp",
          "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose=False):
    """Compile oracle/nmg_oracle.c into oracle/libnmg_oracle.so."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc"] + CFLAGS + ["-shared", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
