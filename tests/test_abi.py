"""The C-ABI library loads and exports every function include/fm.h declares
(CPU only: no compute call)."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1505_07959_amd", "libfm.so")
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")]


def declared():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(fm_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_interface():
    names = declared()
    for f in ("fm_flow_create", "fm_parareal_solve", "fm_fine_propagate", "fm_coarse_propagate", "fm_destroy",
              "fm_last_error"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_declared_symbols():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = declared() - exported
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_loads_and_resolves():
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert getattr(lib, name) is not None
    lib.fm_last_error.restype = ctypes.c_char_p
    assert lib.fm_last_error() == b""
