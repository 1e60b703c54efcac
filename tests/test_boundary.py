"""CPU checks of the C ABI boundary: the library builds, loads and exports
every entry point include/tlim.h declares.  No device call is made."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tlim.h")
LIB = os.path.join(ROOT, "paper_2106_00282_amd", "libtlim.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tlim_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for name in ("tlim_create", "tlim_advance_parabolic", "tlim_set_field", "tlim_get_field", "tlim_adjoint_parabolic"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_2106_00282_amd import build
        build.build()
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    from paper_2106_00282_amd import tlim
    assert sorted(tlim.EXPORTED) == declared_symbols()
    lib = tlim.load_library()
    # host-only calls: status names
    assert lib.tlim_status_str(0) == b"TLIM_OK"
    assert lib.tlim_status_str(5) == b"TLIM_E_NOCONV"


def test_create_rejects_bad_grid_without_device():
    """Argument validation happens before any device query."""
    from paper_2106_00282_amd import tlim
    lib = tlim.load_library()
    g = tlim.Grid()
    for d in range(3):
        g.n[d], g.h[d], g.bc[d] = 4, 0.25, 0
    g.n[1] = 0
    out = ctypes.c_void_p()
    assert lib.tlim_create(ctypes.byref(g), 0, None, ctypes.byref(out)) == tlim.E_ARG
    g.n[1] = 4
    g.bc[2] = 7
    assert lib.tlim_create(ctypes.byref(g), 0, None, ctypes.byref(out)) == tlim.E_ARG
    g.bc[2] = 0
    assert lib.tlim_create(ctypes.byref(g), 3, None, ctypes.byref(out)) == tlim.E_ARG


def test_product_path_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2106_00282_amd import tlim
    monkeypatch.setattr(tlim, "_lib", None)
    with pytest.raises(ImportError):
        tlim.load_library(str(tmp_path / "missing.so"))


def test_binding_holds_no_arithmetic_of_the_method():
    """The Python binding marshals arguments only: it imports no maths
    module and names no function or constant of eq. LIM's schedule
    (P = ceil(pi/4 sqrt(tau lambda + 1)), the Chebyshev roots) or of the
    heat step; workspace sizes come from the library."""
    import ast
    src = open(os.path.join(ROOT, "paper_2106_00282_amd", "tlim.py")).read()
    tree = ast.parse(src)
    imported = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            imported |= {a.name.split(".")[0] for a in node.names}
        elif isinstance(node, ast.ImportFrom):
            imported.add((node.module or "").split(".")[0])
    assert not imported & {"math", "numpy", "cmath", "scipy"}, imported
    names = {n.attr for n in ast.walk(tree) if isinstance(n, ast.Attribute)}
    names |= {n.id for n in ast.walk(tree) if isinstance(n, ast.Name)}
    banned = {"sqrt", "ceil", "cos", "pi", "acos", "floor", "log", "exp", "pow"}
    assert not names & banned, names & banned
    # no operators beyond size bookkeeping (ctypes array types, the
    # checkpoint count) and the unit box's default spacing h = 1/n
    ops = [type(n.op).__name__ for n in ast.walk(tree) if isinstance(n, ast.BinOp)]
    assert set(ops) <= {"Add", "Sub", "Mult", "FloorDiv", "Div"}, set(ops)
    assert sum(op == "Div" for op in ops) == 1


def test_product_does_not_import_oracle():
    """The package never refers to the oracle."""
    pkg = os.path.join(ROOT, "paper_2106_00282_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "oracle" not in text.lower() or fn == "workloads.py", fn


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for more it exits with a message
    before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_ctypes_structs_match_the_header_fields():
    """The binding's structs list the header's fields in order (the ABI is
    by position)."""
    from paper_2106_00282_amd import tlim
    text = open(HEADER).read()

    def fields(struct):
        end = text.index("} " + struct + ";")
        body = text[text.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            # the declarators after the type: the last identifier of each
            first, *more = decl.split(",")
            for d in [first] + more:
                names.append(re.search(r"(\w+)\s*(\[[^\]]*\])?\s*$", d).group(1))
        return names

    for py, struct in ((tlim.Grid, "tlim_grid"), (tlim.Phase, "tlim_phase"), (tlim.StepOptsC, "tlim_step_opts"),
                       (tlim.ReportC, "tlim_step_report"), (tlim.HypOptsC, "tlim_hyp_opts"),
                       (tlim.HypReportC, "tlim_hyp_report")):
        assert [f[0] for f in py._fields_] == fields(struct), struct
