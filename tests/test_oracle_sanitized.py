"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle is plain C called through ctypes; a memory error in it (an
out-of-bounds index, a use after free such as a C model freed while a
stepper still points at it) would otherwise show up only as wrong numbers
or a crash somewhere else.  This test builds the same sources with
-fsanitize=address,undefined and runs the oracle's CPU pins against that
build in a child process with the sanitizer runtime preloaded; any report
ends the child with an error.  Host code only: nothing here touches a GPU.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# the oracle's own pin files (the GPU-free ones), run under the sanitizers
PIN_FILES = ["test_oracle_mesh_ops.py", "test_oracle_expm.py", "test_oracle_phi.py",
             "test_oracle_schemes.py", "test_oracle_adjoint.py", "test_oracle_diagnostics.py",
             "test_oracle_topography.py", "test_oracle_cost_nu.py", "test_oracle_threads.py"]


def _runtime(name):
    r = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_asan_ubsan():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    sys.path.insert(0, ROOT)
    from oracle import build_san
    lib = build_san.build_sanitized()
    env = dict(os.environ)
    env.update({
        "ORC_LIBPATH": lib,
        "LD_PRELOAD": asan + ":" + ubsan,
        # CPython's own allocations are not leaks of the oracle
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    files = [os.path.join(ROOT, "tests", f) for f in PIN_FILES]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu"] + files, cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=1500)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
