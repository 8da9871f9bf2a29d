"""The C++ planner under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, built with g++): every lattice 1..12 x 1..12, bond
dimensions 1..5 and mixed, every order and quadrant split, with the plan's
bookkeeping checked by the driver (tests/native/planner_driver.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_planner_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "planner_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1908_08553_amd", "csrc"),
           os.path.join(ROOT, "tests", "native", "planner_driver.cpp"),
           os.path.join(ROOT, "paper_1908_08553_amd", "csrc", "plan.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                         env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert "fails 0" in run.stdout
