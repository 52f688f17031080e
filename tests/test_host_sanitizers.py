"""The host plan code (plan.cpp, hostmath.cpp) built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer and run on the CPU: plans of several shapes (including an odd
side, c < 1/2 and a 2048-point grid) and the rejected ones, plus checks of the FP64 host
numerics (tests/host_plan_sanitize.cpp).  No HIP call is made."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1412_0781_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_plan_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_plan_sanitize")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__=1", f"-I{ROCM}/include", f"-I{ROOT}/include",
           f"-I{CSRC}", os.path.join(ROOT, "tests", "host_plan_sanitize.cpp"), os.path.join(CSRC, "plan.cpp"),
           os.path.join(CSRC, "hostmath.cpp"), f"-L{ROCM}/lib", "-lamdhip64", "-lpthread", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               LD_LIBRARY_PATH=f"{ROCM}/lib:" + os.environ.get("LD_LIBRARY_PATH", ""))
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-6000:]
    assert "0 failure(s)" in r.stdout
