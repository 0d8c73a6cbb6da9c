"""The C-ABI library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

`tests/host/abi_host.cpp` includes the library source, is built with both sanitizers on its host
code only (the kernels come from the built library, and none runs) and checks the argument
validation of every entry point, the launch plan's layout of random ragged batches (each drop's
elements covered once, offsets as prefix sums, longest-first items), the user-group plans of
drops above 64 users and the Gauss-Legendre table; any sanitizer report fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2503_18118_amd")
LIB = os.path.join(PKG, "libxlmimo.so")
SRC = os.path.join(ROOT, "tests", "host", "abi_host.cpp")


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def test_host_code_under_sanitizers(tmp_path):
    hipcc = _hipcc()
    if hipcc is None or not os.path.exists(LIB):
        pytest.skip("needs hipcc and the built library")
    exe = str(tmp_path / "abi_host")
    cmd = [hipcc, "--offload-arch=gfx950", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(PKG, "csrc"),
           SRC, "-o", exe, "-L" + PKG, "-lxlmimo", "-Wl,-rpath," + PKG]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:alloc_dealloc_mismatch=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "passed" in r.stdout
