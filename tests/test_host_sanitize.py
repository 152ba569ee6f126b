"""The host cluster tree and block partition (csrc/plan.cpp) under
AddressSanitizer and UndefinedBehaviorSanitizer (no GPU): g++ builds
plan.cpp with tests/plan_sanitize_driver.cpp, which builds plans for
ordinary and degenerate point sets (equal points, collinear points,
duplicate clusters, one point) and checks the permutation, offsets and
pair lists; any out-of-bounds access, leak or undefined behaviour ends the
run with a report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_17656_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers (host API types only)")
def test_plan_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-I", "/opt/rocm/include",
           os.path.join(ROOT, "tests", "plan_sanitize_driver.cpp"), os.path.join(CSRC, "plan.cpp"),
           "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    # verify_asan_link_order=0: the environment may preload another library
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, (run.stdout + run.stderr)[-4000:]
    assert "all checks passed" in run.stdout
