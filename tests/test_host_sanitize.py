"""The host-side plan code of the C ABI (api.cpp, tune.cpp, interp.cpp)
built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer (leak
detection on) and driven by tests/host/plan_driver.cpp: plans over every
precision, layout, basis and kernel on a grid of sizes, heterocorrelation,
interpolation weights, batched plans, invalid descriptors and compute calls
that fail validation.  The kernel launchers are link-time stubs
(tests/host/launch_stubs.cpp) that abort if reached.  Needs no GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1808_00685_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")
ROCM = "/opt/rocm"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(os.path.join(ROCM, "lib", "libamdhip64.so")),
                    reason="needs g++ and the HIP runtime library")
def test_plan_code_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "plan_driver")
    srcs = [os.path.join(CSRC, f) for f in ("api.cpp", "tune.cpp", "interp.cpp")]
    srcs += [os.path.join(HOST, f) for f in ("launch_stubs.cpp", "plan_driver.cpp")]
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wno-unused-result",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-D__HIP_PLATFORM_AMD__", "-D__host__=", "-D__device__=",
           "-I" + os.path.join(ROCM, "include"), "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           *srcs, "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-ldl", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ,
               ASAN_OPTIONS="verify_asan_link_order=0:detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1",
               CORR2D_TUNE_TABLE=os.path.join(ROOT, "paper_1808_00685_amd", "tune", "gfx950.tsv"),
               LD_LIBRARY_PATH=os.path.join(ROCM, "lib") + ":" + os.environ.get("LD_LIBRARY_PATH", ""))
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env, cwd=str(tmp_path))
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "all expectations hold" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
