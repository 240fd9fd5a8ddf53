"""CPU regression tests of merge host/device logic: the truncation step with
non-finite singular values, and the TSQR tree's node indexing.

Compiles tests/host/trunc_test.cpp (which includes the library's own trunc.h, the
code the merge kernel runs per workgroup) with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer and runs it: NaN, infinite and huge values must sort
last, never be kept, be reported, and leave a valid permutation and a kept rank in
[0, capacity]."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_truncation_step_under_sanitizers(tmp_path):
    src = os.path.join(ROOT, "tests", "host", "trunc_test.cpp")
    exe = str(tmp_path / "trunc_test")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           src, "-o", exe]
    subprocess.run(cmd, check=True)
    res = subprocess.run([exe], capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "trunc host test ok" in res.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_tsqr_tree_slots_under_sanitizers(tmp_path):
    """Every tree node the merge kernels address fits the slots the host allocates
    (chunk counts that are not powers of two need more than 2n - 1 nodes)."""
    src = os.path.join(ROOT, "tests", "host", "tree_test.cpp")
    exe = str(tmp_path / "tree_test")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    src, "-o", exe], check=True)
    res = subprocess.run([exe], capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "tree host test ok" in res.stdout
