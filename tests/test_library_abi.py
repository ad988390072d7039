"""The C-ABI library loads and exports every symbol declared in include/hdg.h
(no device calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2402_11361_amd", "libhdg.so")


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "hdg.h")).read()
    return sorted(set(re.findall(r"\b(hdg_[a-z_0-9]+)\s*\(", src)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhdg.so not built (run __graft_entry__.build())")
def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    syms = declared_symbols()
    assert "hdg_setup_mesh" in syms and "hdg_fgmres_solve" in syms
    for s in syms:
        assert hasattr(lib, s), s


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhdg.so not built")
def test_binding_declares_same_names():
    from paper_2402_11361_amd import hdg
    assert set(declared_symbols()) == set(hdg.EXPORTS)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhdg.so not built")
def test_status_strings_and_null_checks():
    lib = ctypes.CDLL(LIB)
    lib.hdg_status_string.restype = ctypes.c_char_p
    assert lib.hdg_status_string(0) == b"ok"
    assert lib.hdg_status_string(4) == b"singular local matrix"
    # null arguments are rejected before any device work
    lib.hdg_setup_mesh.restype = ctypes.c_int
    assert lib.hdg_setup_mesh(None, None, None, None) == 1
    lib.hdg_query_sizes.restype = ctypes.c_int
    assert lib.hdg_query_sizes(None, None) == 1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhdg.so not built")
def test_chunk_plan_entry_points_reject_a_null_context():
    lib = ctypes.CDLL(LIB)
    n = ctypes.c_int(0)
    for name, args in [("hdg_set_chunking", (None, 2)), ("hdg_set_chunk_buffers", (None, 2)),
                       ("hdg_set_factor_store", (None, 4, 1)), ("hdg_factor_store_macros", (None, ctypes.byref(n))),
                       ("hdg_set_progress", (None, 1))]:
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        assert f(*args) == 1, name  # HDG_EINVAL
