"""Host-side checks of the benchmark's contract and of its byte accounting (no GPU)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


@pytest.mark.parametrize("precision,w", [("fp64", 8), ("mixed", 4)])
def test_algorithmic_bytes_per_cell(precision, w):
    """The per-cell bytes stated for each grid kernel: operator A reads z, p_old, diag
    (+ tx, ty with cellwise conductances, + tz in 3-D) and writes p_new, q; update B reads
    x, p, r, q, writes x, r and z (block IC(0) and the V-cycle add the FP32 pivots and
    conductances); P (V-cycle finest level) reads z_p, r, a quarter word of the coarse
    correction and FP32 coefficients, writes z."""
    g = bench.grid_bytes_per_cell
    assert g("A", precision, "mg", True) == 7 * w
    assert g("A", precision, "mg", False) == 5 * w
    assert g("A", precision, "bic0", True, dim=3) == 8 * w
    assert g("B", precision, "mg", True) == 7 * w + 12
    assert g("B", precision, "jacobi", True) == 7 * w
    assert g("P", precision, "mg", True) == 3 * w + w / 4 + 16
    assert g("P", precision, "mg", False) == 3 * w + w / 4 + 8
    # fused with the restriction into level 1: + FP32 diagonal, a quarter word of r_c and
    # the block edges (two words and 4 B per 64 cells)
    assert g("B", precision, "mg", True, fused=True) == 7 * w + 16 + w / 4 + (2 * w + 4) / 64


def test_roofline_from_samples():
    """A dominant kernel is the one with the most estimated time; working launches are the
    issued ones scaled by the working share of the samples; achieved = bytes / time."""
    kind_time = {"A": (10, 5.0, 100, 8, 4.8), "B": (10, 2.0, 100, 10, 2.0)}
    tot = {"A": 80 * 1e9, "B": 100 * 1e9}
    dom, other = bench.roofline(kind_time, tot, "fp64", "mg", "C2")
    assert dom["kernel"].startswith("k_pcg_A") and len(other) == 1
    # A: 80 working launches of 0.6 ms carrying 1e9 bytes each
    assert np.isclose(dom["avg_launch_us"], 600.0)
    assert np.isclose(dom["algorithmic_bytes_per_launch"], 1e9)
    assert np.isclose(dom["achieved"], 1e9 / 0.6e-3 / 1e9)
    assert np.isclose(dom["frac"], dom["achieved"] / 8000.0)


def test_vcycle_levels_and_bytes():
    """A 2048 x 2048 grid coarsens 2048^2 -> 1024^2 -> ... -> 16^2 (<= 256 cells); levels of at
    most 1024 cells form the tail.  Restriction + pre-smoothing and post-smoothing run on
    every level above the tail: RS moves (2 words + 12 B) per cell of the finer level
    (4 B at a finest level without conductance arrays) and (2 words + 12 B) per coarse
    cell; PC moves 3 words + w / 4 + 16 B per cell; R (into the tail) the finer level's
    2 words + 12 B and one coarse word per cell.  A hierarchy cut after 3 levels has no
    tail."""
    lv = bench.mg_levels(2048, 2048)
    assert [a for a, _ in lv] == [2048, 1024, 512, 256, 128, 64, 32, 16]
    n = [a * a for a, _ in lv]
    b = bench.vcycle_bytes(2048, 2048, "fp64", True)
    rs = sum(n[l - 1] * 28 + n[l] * 28 for l in range(1, 6))
    pc = sum(n[l] * 42 for l in range(1, 6))
    assert np.isclose(b["RS"], rs) and np.isclose(b["PC"], pc)
    assert np.isclose(b["R"], n[5] * 28 + n[6] * 8) and b["TAIL"] == 0
    b3 = bench.vcycle_bytes(2048, 2048, "fp64", False, nlev=3)
    assert np.isclose(b3["RS"], n[0] * 20 + n[1] * 28 + sum(n[l - 1] * 28 + n[l] * 28
                                                          for l in (2, 3)))
    assert b3["R"] == 0
    # fused: level 1 reads and writes r_c, writes z_p, reads its factor, plus one fine edge
    # row in 8 (a word and 4 B per fine column) and 3 edge columns per 128 fine columns
    bf = bench.vcycle_bytes(2048, 2048, "fp64", True, nlev=3, fused=True)
    assert np.isclose(bf["RS"], n[1] * (36 + 6 + 24 * 12 / 256)
                      + sum(n[l - 1] * 28 + n[l] * 28 for l in (2, 3)))
    assert bench.mg_fused(2048, 2048) and not bench.mg_fused(64, 64)
    assert not bench.mg_fused(2048, 2048, dim=3) and not bench.mg_fused(2048, 2048, nlev=0)
    assert not bench.mg_fused(2048, 2048, precision="mixed")
    w = bench.working_launches([[7, 3], [5, 9]], "mg", [3, 6], [(2048, 2048), (2048, 2048)])
    # 7 + 9 iterations; 5 levels above the tail in the deeper hierarchy, which has a tail
    assert w["A"] == 16 and w["RS"] == 16 * 5 and w["TAIL"] == 16 and w["R"] == 16
    # a truncated last level smoothed once has no post-smoothing launch or bytes
    b1 = bench.vcycle_bytes(2048, 2048, "fp64", True, nlev=3, once=True)
    b2 = bench.vcycle_bytes(2048, 2048, "fp64", True, nlev=3)
    assert np.isclose(b2["PC"] - b1["PC"], n[3] * 42) and b1["RS"] == b2["RS"]
    w1 = bench.working_launches([[6]], "mg", [3], [(2048, 2048)], [True])
    assert w1["RS"] == 18 and w1["PC"] == 12 and w1["TAIL"] == 0
