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
