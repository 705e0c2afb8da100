"""The host runtime (runtime.cpp, runtime_fdm.cpp, runtime_program.cpp) built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer, with the HIP runtime acting on host memory and
every kernel launcher replaced by a check that the buffers the kernel would touch lie inside the
caller's allocations (tests/host_sanitize/stubs.cpp).  The driver (tests/host_sanitize/driver.cpp)
walks every entry point over a sweep of shapes (n, r, dtype, Kraus count, fused and plain form):
workspace sizing and carving, gate passes, chained compressions, outputs, records and the
reverse-sweep calls, the program-level calls, the full-rank comparator, a batch, and the argument
checks.  Passing means no sanitizer report, no leak and no kernel region outside its buffer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2009_06657_amd", "csrc")
HS = os.path.join(ROOT, "tests", "host_sanitize")


def test_host_runtime_under_asan_and_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"):
        pytest.skip("g++ or the HIP headers are missing")
    exe = str(tmp_path / "hsan")
    cmd = [gxx, "-O1", "-g", "-std=c++20", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(CSRC, "runtime.cpp"), os.path.join(CSRC, "runtime_fdm.cpp"),
           os.path.join(CSRC, "runtime_program.cpp"), os.path.join(HS, "stubs.cpp"), os.path.join(HS, "driver.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=900)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout + r.stderr)[-6000:]
    assert "regions outside their buffers 0, failed expectations 0" in r.stdout
