"""NLMC host bookkeeping (no GPU): coarse units, the oversampled regions' banded local
orderings and band widths, the region unit lists and the unit pairs whose basis functions
interact, recounted by brute force on random fracture networks by a C++ self-test built
with g++ (with AddressSanitizer and UBSan when the toolchain has them)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "tests", "nlmc_plan_selftest.cpp"),
       os.path.join(ROOT, "paper_2209_01158_amd", "csrc", "nlmc_host.cpp")]


def _build(tmp_path, sanitize):
    exe = str(tmp_path / ("plan_san" if sanitize else "plan"))
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall"]
    if sanitize:
        cmd += ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    cmd += SRC + ["-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    return exe if res.returncode == 0 else None, res.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_nlmc_plan_selftest(tmp_path):
    exe, err = _build(tmp_path, sanitize=True)
    if exe is None:
        exe, err = _build(tmp_path, sanitize=False)
    assert exe, err
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0 and res.stdout.strip().endswith("OK"), res.stdout + res.stderr
