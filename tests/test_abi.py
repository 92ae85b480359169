"""CPU checks of the C ABI: the library builds, loads, and exports every entry point that
include/rrq.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

from paper_2411_08342_amd import rrq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rrq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rrq_[a-z_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared_functions()
    assert set(rrq.EXPORTED) == set(names), names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(rrq.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(rrq.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_status_strings():
    if not os.path.exists(rrq.LIB_PATH):
        pytest.skip("library not built")
    L = rrq.lib()
    assert L.rrq_status_string(0) == b"ok"
    assert L.rrq_status_string(-1) == b"invalid argument"


def test_argument_errors_return_before_launch():
    """Null arguments are rejected on the host with RRQ_ERR_ARG, without touching a GPU."""
    if not os.path.exists(rrq.LIB_PATH):
        pytest.skip("library not built")
    L = rrq.lib()
    out = ctypes.c_void_p()
    assert L.rrq_plan_create(None, None, None, ctypes.byref(out)) == -1
    s = rrq.Surface()
    s.npatch = 0
    assert L.rrq_plan_create(ctypes.byref(s), None, None, ctypes.byref(out)) == -1
    assert L.rrq_plan_destroy(None) == -1
    assert L.rrq_assemble(None, None, 15, 0, None, None, None, None, 0, None, None, None, 0, None,
                          None) == -1
    assert L.rrq_weights_size(None, None, None, None) == -1
    assert L.rrq_plan_patch_flags(None, 0.0, None, None) == -1
    assert L.rrq_assemble_noalloc(None, None, 15, 0, None, None, None, None, 0, None, None,
                                  None) == -1


def test_status_strings_cover_every_code():
    if not os.path.exists(rrq.LIB_PATH):
        pytest.skip("library not built")
    L = rrq.lib()
    for code in range(-7, 1):
        assert L.rrq_status_string(code) != b"unknown status", code
