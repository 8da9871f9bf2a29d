"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (built
with g++, no device code):

* the C++ planner: every lattice 1..12 x 1..12, bond dimensions 1..5 and
  mixed, every order and quadrant split, with the plan's bookkeeping checked,
  and every column-sweep cut plan (cached environments: same steps as the
  full sweep, seed and rescale slots, left and right cuts ending in the same
  bonds) (tests/native/planner_driver.cpp);
* the served loop's admission arena (first fit with coalescing): randomized
  alloc/release against a brute-force model (tests/native/arena_driver.cpp).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1908_08553_amd", "csrc")
FLAGS = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build_and_run(tmp_path, sources):
    exe = str(tmp_path / "driver")
    subprocess.run(FLAGS + sources + ["-o", exe], check=True, capture_output=True, timeout=300)
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                         env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert "fails 0" in run.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_planner_clean_under_sanitizers(tmp_path):
    build_and_run(tmp_path, [os.path.join(ROOT, "tests", "native", "planner_driver.cpp"),
                             os.path.join(CSRC, "plan.cpp")])


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_arena_first_fit_against_model(tmp_path):
    build_and_run(tmp_path, [os.path.join(ROOT, "tests", "native", "arena_driver.cpp")])
