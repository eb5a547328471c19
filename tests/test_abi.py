"""The C-ABI library loads without a GPU and exports what include/sfcnl.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfcnl.h")
LIB = os.path.join(ROOT, "paper_2602_19873_amd", "libsfcnl.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\s*\*)\s*(\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libsfcnl.so missing: run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_header_declares_the_paths_calls():
    names = _declared()
    for n in ("sfc_sort", "sfc_gather", "build_clusters", "build_nlist", "nlist_pass", "nlist_decode",
              "sfcnl_create", "sfcnl_destroy"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_header():
    from paper_2602_19873_amd import _lib
    assert sorted(_lib.SYMBOLS) == _declared()


def test_workspace_queries_are_host_only(lib):
    from paper_2602_19873_amd import _lib
    L = _lib.load()
    b = ctypes.c_size_t()
    assert L.sfc_sort_workspace(0, ctypes.byref(b)) == 0
    small = b.value
    assert L.sfc_sort_workspace(1 << 20, ctypes.byref(b)) == 0
    assert b.value > small + 12 * (1 << 20)
    o = _lib.NlistOpts(8, 1, 64, 512)
    assert L.build_nlist_workspace(100000, ctypes.byref(o), ctypes.byref(b)) == 0
    assert b.value > 100000 // 64 * 512 * 5
    for bad in (_lib.NlistOpts(5, 1, 64, 512), _lib.NlistOpts(8, 2, 64, 512), _lib.NlistOpts(8, 1, 4, 512),
                _lib.NlistOpts(8, 1, 64, 0), _lib.NlistOpts(8, 1, 64, 512, 2),
                _lib.NlistOpts(8, 1, 64, 512, 0, (ctypes.c_float * 3)(1.0, -1.0, 0.0)),
                _lib.NlistOpts(8, 1, 64, 512, 0, (ctypes.c_float * 3)(float("inf"), 0.0, 0.0))):
        assert L.build_nlist_workspace(1000, ctypes.byref(bad), ctypes.byref(b)) == _lib.E_ARG
    assert L.sfc_sort_workspace(-1, ctypes.byref(b)) == _lib.E_ARG
    ok = _lib.NlistOpts(8, 1, 64, 512, 1, (ctypes.c_float * 3)(1.0, 0.0, 2.5))
    assert L.build_nlist_workspace(1000, ctypes.byref(ok), ctypes.byref(b)) == 0


def test_null_context_rejected(lib):
    from paper_2602_19873_amd import _lib
    L = _lib.load()
    assert L.sfcnl_sync(None) == _lib.E_ARG
    assert L.sfc_sort(None, 10, None, None, None, None, None, None, None, 0) == _lib.E_ARG
    assert L.nlist_pass(None, 10, 8, 1, 0, None, None, None, None, None, None, None, None, None, None) == _lib.E_ARG
    par = _lib.LjParams(1.0, 0.01, 0.0, 0.05)
    assert L.nlist_pass_lj(None, 10, 8, 1, 0, None, None, None, None, None, None, ctypes.byref(par), None, None,
                           None, None, None) == _lib.E_ARG
    assert L.sfcnl_version().startswith(b"sfcnl")


def test_rows_calls_are_checked(lib):
    from paper_2602_19873_amd import _lib
    L = _lib.load()
    b = ctypes.c_size_t()
    assert L.build_rows_workspace(1000, ctypes.byref(b)) == 0 and b.value >= 8 * 1000
    assert L.build_rows_workspace(-1, ctypes.byref(b)) == _lib.E_ARG
    used = ctypes.c_size_t()
    assert L.build_rows(None, 10, 8, 1, None, None, None, None, None, None, 1, None, None, 0, None, None, 0,
                        ctypes.byref(used)) == _lib.E_ARG
    assert L.rows_pass(None, 10, 1, None, None, None, None, None, None, None, None, None, None) == _lib.E_ARG
