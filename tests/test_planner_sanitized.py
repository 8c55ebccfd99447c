"""The tile planner (host-only C++) built with AddressSanitizer and
UndefinedBehaviorSanitizer and run over random 2D and 3D chains, tile
heights, slot counts and capacities (tests/planner_sanitize.cpp): any memory
error or undefined behaviour aborts it, and every plan must keep the tiling's
invariants."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_planner_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "planner_sanitize")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-o", exe,
           os.path.join(HERE, "planner_sanitize.cpp"),
           os.path.join(ROOT, "paper_1709_02125_amd", "csrc", "planner.cpp")]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, "300"], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout, r.stderr[-3000:])
    assert r.returncode == 0, r.stderr[-3000:]
    assert "failures 0" in r.stdout
