"""CPU checks of the boundary: libdade.so loads and exports every entry point that
include/dade.h declares; the product package never reaches the oracle."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dade.h")
PKG = os.path.join(ROOT, "paper_2411_17229_amd")


def declared():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return sorted(set(re.findall(r"\b(dade_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for required in ("dade_build_index", "dade_rotate", "dade_calibrate", "dade_search"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2411_17229_amd import dade
    if not os.path.exists(dade.LIB_PATH):
        pytest.skip("libdade.so not built")
    L = ctypes.CDLL(dade.LIB_PATH)
    for name in declared():
        assert hasattr(L, name), name
    assert set(declared()) == set(dade.EXPORTED)


def test_binding_names_match_the_c_entry_points():
    from paper_2411_17229_amd import dade
    for name in declared():
        assert callable(getattr(dade, name)), name


def test_product_code_never_touches_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", src, re.M), f
                assert "oracle" not in src.lower() or f.endswith(".py") and "oracle" not in \
                    re.sub(r'""".*?"""|#.*', "", src, flags=re.S).lower(), f


def test_serve_rejects_missing_arguments_before_touching_a_device():
    """dade_serve validates its handle and options before any HIP call (safe without a GPU)."""
    from paper_2411_17229_amd import dade
    if not os.path.exists(dade.LIB_PATH):
        pytest.skip("libdade.so not built")
    L = dade.lib()
    args = [None] * 13
    args[1] = 0
    assert L.dade_serve(*args) == dade.DADE_EINVAL
    assert "index is NULL" in dade.dade_last_error()


def test_new_entry_points_reject_null_handles_before_touching_a_device():
    """dade_autotune, dade_graph_build, dade_graph_search and dade_graph_export validate their
    handle before any HIP call (safe without a GPU)."""
    from paper_2411_17229_amd import dade
    if not os.path.exists(dade.LIB_PATH):
        pytest.skip("libdade.so not built")
    L = dade.lib()
    assert L.dade_autotune(None, None, 1, 10, 8, None, None, 0.5, 1, None, None, None, None) == dade.DADE_EINVAL
    assert L.dade_graph_build(None, 16, 8, 4, 0, None) == dade.DADE_EINVAL
    assert L.dade_graph_search(None, None, 1, 10, 32, 4, 0, None, None, None, None) == dade.DADE_EINVAL
    assert L.dade_graph_export(None, None, None, None) == dade.DADE_EINVAL
    assert "NULL" in dade.dade_last_error()


def _c_layout(struct, fields):
    """sizeof and field offsets of a struct of include/dade.h, from a C program built with gcc."""
    import subprocess
    import tempfile
    body = "\n".join(f'  printf("%zu ", offsetof({struct}, {f}));' for f in fields)
    prog = (f'#include <stddef.h>\n#include <stdio.h>\n#include "dade.h"\nint main(void) {{\n'
            f'  printf("%zu ", sizeof({struct}));\n{body}\n  return 0;\n}}\n')
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        open(src, "w").write(prog)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        return [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]


@pytest.mark.parametrize("struct,cls", [("dade_search_opts", "SearchOpts"), ("dade_search_record", "SearchRecord"),
                                        ("dade_tune_result", "TuneResult"),
                                        ("dade_serve_opts", "ServeOpts"), ("dade_times", "Times")])
def test_binding_structs_match_the_header_layout(struct, cls):
    """The ctypes mirrors of the option and record structs have the C layout field for field (the
    search record carries Delta_d, the schedule, the rerank rule and the nprobe clamp)."""
    import shutil
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    from paper_2411_17229_amd import dade
    c = getattr(dade, cls)
    names = [f for f, _ in c._fields_]
    layout = _c_layout(struct, ["lambda" if n == "lambda_" else n for n in names])
    assert layout[0] == ctypes.sizeof(c)
    assert layout[1:] == [getattr(c, n).offset for n in names]
