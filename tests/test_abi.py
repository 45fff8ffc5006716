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


def test_binding_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of fm_problem, fm_params and fm_stats have the sizes
    and field offsets the C compiler gives the header's structs."""
    import ctypes
    import shutil
    import subprocess
    import ast
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    fields = {"fm_params": ["T", "N", "fine_steps", "tol", "refine_tol", "fine_method", "variant"],
              "fm_stats": ["iters", "increment", "hist", "fine_launches", "fine_phase_ms", "basis_size"],
              "fm_problem": ["kind", "n", "A", "lda"]}
    prog = ["#include <stdio.h>", "#include <stddef.h>", '#include "fm.h"', "int main(void) {"]
    for st, fs in fields.items():
        prog.append('printf("%%zu\\n", sizeof(%s));' % st)
        for f in fs:
            prog.append('printf("%%zu\\n", offsetof(%s, %s));' % (st, f))
    prog.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(prog))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I" + os.path.join(root, "include"), str(c), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    src = open(os.path.join(root, "paper_1505_07959_amd", "fm.py")).read()
    tree = ast.parse(src)
    ns = {}
    body = [n for n in tree.body if isinstance(n, ast.ClassDef) and n.name in fields]
    exec(compile(ast.Module(body=body, type_ignores=[]), "fm_structs", "exec"), {"ctypes": ctypes}, ns)
    want = []
    for st, fs in fields.items():
        cls = ns[st]
        want.append(ctypes.sizeof(cls))
        for f in fs:
            want.append(getattr(cls, f).offset)
    assert got == want
