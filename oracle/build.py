"""Build the oracle library (test infrastructure only).

Compiles the plain C reference with gcc: no fast-math and no FMA contraction,
so every FP64 operation is the IEEE operation written in the source.  OpenMP
only distributes independent faces and cells; results do not depend on the
thread count.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liborc.so")
SOURCES = ["hydro_oracle.c", "exact_riemann.c"]
FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
         "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force=True, extra_flags=()):
    """Compile liborc.so in place; with force=False, only if it is missing."""
    if not force and os.path.exists(LIB):
        return LIB
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = ["gcc", *FLAGS, *extra_flags, "-o", tmp, *srcs, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, extra_flags=sys.argv[1:]))
