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
    assert L.dade_graph_build(None, None, 16, 8, 4, None) == dade.DADE_EINVAL
    assert L.dade_graph_search(None, None, 1, 10, 32, 4, 0, None, None, None, None) == dade.DADE_EINVAL
    assert L.dade_graph_export(None, None, None, None) == dade.DADE_EINVAL
    assert "NULL" in dade.dade_last_error()
