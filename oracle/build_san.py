"""Sanitizer build of the CPU oracle (test infrastructure only): the same
sources under AddressSanitizer and UndefinedBehaviorSanitizer, host code
compiled by gcc, for the CPU test that runs the oracle's pins against it."""
import os
import subprocess

from .build import HERE, SOURCES

SAN_LIB = os.path.join(HERE, "liboracle_san.so")


def build_sanitized(verbose=False):
    """Serial build (the parallel-loop pragmas are ignored)."""
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           "-Wno-unknown-pragmas", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-o", SAN_LIB] + \
          [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return SAN_LIB
