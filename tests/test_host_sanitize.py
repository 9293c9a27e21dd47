"""The plan builder's host code under AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer (CPU only).

csrc/plan.cpp -- argument checks, element validation (ids, repeats, volume,
finite coordinates), Morton reordering, the slot-packed incidence lists and
neighbour lists, the settings and their bounds, and the clean-up after every
allocation failure -- is compiled with g++ and the sanitizers against host-memory
stand-ins for the HIP runtime calls it makes (tests/host_sanitize/hip_stub.cpp),
and driven through its C entry points by tests/host_sanitize/plan_driver.cpp.
The run must report every case as expected, with no sanitizer report and no
leak (each allocation of a plan is made to fail in turn)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(ROOT, "paper_2308_08410_amd", "csrc", "plan.cpp"),
       os.path.join(HERE, "host_sanitize", "hip_stub.cpp"),
       os.path.join(HERE, "host_sanitize", "plan_driver.cpp")]
FLAGS = ["-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
         "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2308_08410_amd", "csrc")]


def test_plan_builder_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path / "plan_asan")
    b = subprocess.run([gxx, *FLAGS, *SRC, "-o", exe], capture_output=True, text=True, timeout=300)
    if b.returncode != 0 and "asan" in b.stderr.lower() and "cannot find" in b.stderr.lower():
        pytest.skip("no sanitizer runtime: " + b.stderr[-200:])
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0 and "OK (0 failures)" in r.stdout, out[-4000:]
