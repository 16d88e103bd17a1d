"""Build the HIP library in-tree for gfx950 (hipcc, no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmcdec.so")
SOURCES = [os.path.join(HERE, "csrc", f)
           for f in ("engine.hip", "nlmc.hip", "host_setup.cpp", "nlmc_host.cpp", "scheduler.cpp",
                     "server.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # no packed FP32 instructions in any generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"),
         # dense SPD inverse of the crossing-cell Schur complement at setup
         "-lrocsolver", "-lrocblas"]


def build(verbose: bool = False) -> str:
    srcs = [s for s in SOURCES if os.path.exists(s)]
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + srcs + ["-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libmcdec.so")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
