"""Compile the CPU oracle into oracle/liboracle.so (plain gcc, -O2, no
fast-math; OpenMP only for the independent cell loops, one thread unless
orc_set_threads asks for more).  Test infrastructure only."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["orc_swe.c", "orc_linalg.c", "orc_phi.c", "orc_schemes.c", "orc_adjoint.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-Wall",
           "-Wno-unused-function", "-o", LIB] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
