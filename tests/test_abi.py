"""The C-ABI library loads on a machine without a GPU and exports every
entry point that include/we.h declares.  No compute call is made."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "we.h")
LIB = os.path.join(ROOT, "paper_1303_5986_amd", "libwe.so")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"WE_API\s+[\w\s\*]+?\b(we_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for core in ("we_create_network", "we_init", "we_step_intervals", "we_histogram", "we_mfpt"):
        assert core in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libwe.so not built")
    lib = ctypes.CDLL(LIB)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_binding_declares_every_symbol():
    from paper_1303_5986_amd import we
    assert sorted(we.EXPORTED) == declared_symbols()


def test_last_error_callable_without_device():
    if not os.path.exists(LIB):
        pytest.skip("libwe.so not built")
    lib = ctypes.CDLL(LIB)
    lib.we_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.we_last_error(), bytes)
