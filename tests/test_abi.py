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
    assert lib.lp_query_static(None, None, 0, 1, 256, 10, 0.0, None, None, None, None) == 1
    assert lib.lp_fingerprint(None, 256, None, None) == 1
    assert lib.lp_graph_destroy(None) == 0


def test_measures_table_matches_header():
    text = open(HEADER).read()
    for i, m in enumerate(lp.MEASURES):
        assert re.search(rf"LP_{m}\s*=\s*{i}\b", text), m


def test_tuning_struct_matches_header(lib):
    """The binding's lp_tuning mirror has the header's fields, in order."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\} lp_tuning;", text, re.S).group(1)
    want = [(name, int(n) if n else 1) for name, n in re.findall(r"int64_t\s+(\w+)(?:\[(\d+)\])?;", body)]
    got = [(name, getattr(t, "_length_", 1)) for name, t in lp._Tuning._fields_]
    assert want == got
    assert ctypes.sizeof(lp._Tuning) == 8 * sum(n for _, n in want)
    assert lib.lp_set_tuning(None, None) == 1


def test_bucket_defaults_match_header():
    text = open(HEADER).read()
    m = re.search(r"bucket_max\[b\].*?\(defaults ([\d, ]+),", text, re.S)
    assert m is not None
    assert tuple(int(x) for x in m.group(1).replace(" ", "").split(",")) == lp.BUCKET_MAX_DEFAULT
