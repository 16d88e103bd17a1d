"""The C-ABI library loads and exports every function include/mcdec.h declares (no GPU
call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2209_01158_amd", "libmcdec.so")
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


def declared():
    names = set()
    for h in HEADERS:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(mc_\w+)\s*\(", txt))
    return sorted(names)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    names = declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "mcdec_src", os.path.join(ROOT, "paper_2209_01158_amd", "mcdec.py"))
    src = open(spec.origin).read()
    for n in declared():
        assert n in src, f"binding does not wrap {n}"


STRUCTS = {"OmegaDesc": "mc_omega_desc", "ProblemDesc": "mc_problem_desc",
           "Options": "mc_options", "Report": "mc_report", "Info": "mc_info",
           "ServerConfig": "mc_server_config", "RequestInfo": "mc_request_info",
           "ServerStats": "mc_server_stats", "NlmcInfo": "mc_nlmc_info"}


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_struct_layout_matches_header(tmp_path):
    """Every ctypes mirror has the size and field offsets the C compiler gives the header's
    struct (a field added on one side only shifts everything after it)."""
    import subprocess
    from paper_2209_01158_amd import mcdec
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mcdec.h"', 'int main(void) {']
    for py, c in STRUCTS.items():
        cls = getattr(mcdec, py)
        lines.append(f'  printf("{py} size %zu\\n", sizeof({c}));')
        for f in cls._fields_:
            lines.append(f'  printf("{py} {f[0]} %zu\\n", offsetof({c}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    for line in out.splitlines():
        py, field, val = line.split()
        cls = getattr(mcdec, py)
        got = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(val), (py, field, got, val)
