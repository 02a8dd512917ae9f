"""Compiling and running the host builds of HIP kernels under tests/hostbuild
(g++, AddressSanitizer, UndefinedBehaviorSanitizer, no contraction)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOSTBUILD = os.path.join(ROOT, "tests", "hostbuild")


def compile_harness(name: str, out_dir) -> str:
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = os.path.join(str(out_dir), name)
    cmd = [gxx, "-std=c++20", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-ffp-contract=off", "-pthread", "-I", HOSTBUILD,
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2205_14330_amd", "csrc"),
           "-x", "c++", os.path.join(HOSTBUILD, name + ".cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def run(exe, d, mode, arrays, *args):
    """Writes arrays as raw files DIR/<name>.bin and runs the harness."""
    for name, a in arrays.items():
        np.ascontiguousarray(a).tofile(os.path.join(str(d), name + ".bin"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, mode, str(d)] + [str(a) for a in args], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
