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


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_invalid_arguments_are_refused_before_any_device_call():
    """The entry points check their host arguments first: an empty batch, an
    order outside [1, 16384], a leading dimension below n, a NULL matrix, a
    nonzero reserved field, an unknown dtype or flow kind, and a NULL flow
    handle are refused with FM_ERR_INVALID (-1) and a message, before any HIP
    call (so this runs without a GPU); fm_destroy accepts NULL."""
    lib = ctypes.CDLL(LIB)

    class Problem(ctypes.Structure):  # fm_problem (layout checked against the header above)
        _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("n", ctypes.c_int64),
                    ("A", ctypes.c_void_p), ("lda", ctypes.c_int64)]

    P, PP = ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)
    lib.fm_flow_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(Problem), ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_char_p, P]
    lib.fm_flow_create.restype = ctypes.c_int32
    lib.fm_last_error.restype = ctypes.c_char_p
    lib.fm_destroy.argtypes = [P]
    lib.fm_destroy.restype = None
    INVALID, HOMOTOPY, LINEAR, F64, BF16X3 = -1, 1, 5, 0, 4
    buf = (ctypes.c_double * 4)()
    addr = ctypes.addressof(buf)

    def create(problems, batch=None, dtype=F64, out=True):
        arr = (Problem * max(1, len(problems)))(*problems)
        h = P()
        st = lib.fm_flow_create(ctypes.byref(h) if out else None, arr, len(problems) if batch is None else batch,
                                dtype, None, None)
        return st, lib.fm_last_error().decode(), h

    ok = Problem(HOMOTOPY, 0, 2, addr, 2)
    cases = [
        (dict(problems=[ok], batch=0), "batch 0"),
        (dict(problems=[ok], batch=-3), "batch -3"),
        (dict(problems=[ok], dtype=BF16X3 + 1), "unknown dtype"),
        (dict(problems=[ok], dtype=-1), "unknown dtype"),
        (dict(problems=[Problem(LINEAR + 1, 0, 2, addr, 2)]), "unknown flow kind"),
        (dict(problems=[Problem(HOMOTOPY - 1, 0, 2, addr, 2)]), "unknown flow kind"),
        (dict(problems=[Problem(HOMOTOPY, 0, 0, addr, 2)]), "1 <= n <= 16384"),
        (dict(problems=[Problem(HOMOTOPY, 0, 16385, addr, 16385)]), "1 <= n <= 16384"),
        (dict(problems=[Problem(HOMOTOPY, 0, 4, addr, 3)]), "lda >= n"),
        (dict(problems=[Problem(HOMOTOPY, 0, 2, None, 2)]), "A != NULL"),
        (dict(problems=[Problem(HOMOTOPY, 1, 2, addr, 2)]), "reserved == 0"),
        (dict(problems=[ok, Problem(HOMOTOPY, 0, 0, addr, 2)]), "problem 1"),
        (dict(problems=[ok], out=False), "non-NULL"),
    ]
    for kw, msg in cases:
        st, err, h = create(**kw)
        assert st == INVALID and msg in err, (kw, st, err)
        assert not h.value
    # a NULL flow handle is refused by every entry point that takes one
    lib.fm_parareal_solve.argtypes = [P, PP, PP, P, P, P]
    lib.fm_fine_propagate.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, PP, PP, P]
    lib.fm_coarse_propagate.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                        PP, PP, P]
    for f in (lib.fm_parareal_solve, lib.fm_fine_propagate, lib.fm_coarse_propagate):
        f.restype = ctypes.c_int32
    assert lib.fm_parareal_solve(None, None, None, None, None, None) == INVALID
    assert "NULL" in lib.fm_last_error().decode()
    assert lib.fm_fine_propagate(None, 1.0, 0.0, 1, None, None, None) == INVALID
    assert lib.fm_coarse_propagate(None, 1.0, 0.0, 1, 0, None, None, None) == INVALID
    lib.fm_destroy(None)
