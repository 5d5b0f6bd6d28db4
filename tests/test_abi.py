"""CPU checks of the C ABI: the library builds, loads, and exports every symbol
that include/rst.h declares (no compute calls; no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2603_11645_amd as rst

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rst.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rst_[a-z_0-9]+)\s*\(", text)))


def test_header_declarations_match_binding_list():
    assert declared_symbols() == sorted(rst.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(rst.LIB_PATH):
        from paper_2603_11645_amd import _build
        _build.build()
    lib = ctypes.CDLL(rst.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", rst.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (rst_\w+)", out))
    assert set(declared_symbols()) <= exported


def test_status_strings_without_device():
    lib = rst.load_library()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.rst_status_string(code)
    assert b"unknown" in lib.rst_status_string(42)


def test_create_without_device_is_an_error_not_a_crash():
    """rst_create on a machine without a usable device returns a status."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    lib = rst.load_library()
    h = ctypes.c_void_p()
    rc = lib.rst_create(ctypes.byref(h), 0, None)
    assert rc != 0


def test_null_arguments_rejected_before_device_work():
    lib = rst.load_library()
    assert lib.rst_create(None, 0, None) == rst.RST_E_INVAL
    g = rst.rst_csr(10, 0, 4, None, None)
    assert lib.rst_spanning_tree(None, ctypes.byref(g), 0, 0, None, None) == rst.RST_E_INVAL
    assert lib.rst_components(None, ctypes.byref(g), None, None) == rst.RST_E_INVAL
    assert lib.rst_list_rank(None, 4, None, None) == rst.RST_E_INVAL
    lib.rst_destroy(None)
