"""The C-ABI library: loads, exports every symbol include/lp.h declares, and
rejects bad arguments on the host before touching a device.  CPU only."""
import ctypes
import os
import re

import pytest

import paper_2401_11415_amd as lp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lp_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lp.library_path()):
        pytest.fail("liblp.so is not built (run __graft_entry__.build())")
    return lp.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("lp_graph_create", "lp_graph_destroy", "lp_predict", "lp_query",
                 "lp_fingerprint", "lp_status_string", "lp_last_error"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code, name in enumerate(["LP_OK", "LP_ERR_INVALID_ARGUMENT", "LP_ERR_INVALID_GRAPH",
                                 "LP_ERR_OUT_OF_MEMORY", "LP_ERR_DEVICE", "LP_ERR_BUSY"]):
        assert lib.lp_status_string(code).decode() == name


def test_host_side_argument_errors(lib):
    h = ctypes.c_void_p()
    off = (ctypes.c_int64 * 2)(0, 0)
    assert lib.lp_graph_create(-1, off, None, 0, ctypes.byref(h)) == 1
    assert "n must be" in lib.lp_last_error().decode()
    assert lib.lp_graph_create(1, None, None, 0, ctypes.byref(h)) == 1
    assert lib.lp_graph_create(1, off, None, 0, None) == 1
    assert lib.lp_graph_create(1, off, None, 0x80, ctypes.byref(h)) == 1
    cnt = ctypes.c_int64(7)
    assert lib.lp_predict(None, 1, 256, 10, 0.0, None, None, None, ctypes.byref(cnt), None) == 1
    assert cnt.value == 0
    assert lib.lp_query(None, None, 0, 1, 256, 10, 0.0, None, None, None, None) == 1
    assert lib.lp_fingerprint(None, 256, None, None) == 1
    assert lib.lp_graph_destroy(None) == 0


def test_measures_table_matches_header():
    text = open(HEADER).read()
    for i, m in enumerate(lp.MEASURES):
        assert re.search(rf"LP_{m}\s*=\s*{i}\b", text), m
