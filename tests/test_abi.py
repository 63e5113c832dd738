"""The C-ABI boundary without a GPU: the shared library loads, exports every
function include/dgx.h declares (C linkage, unmangled), and the Python
binding wraps each of them under the same name.  No compute call is made.
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgx.h")
LIB = os.path.join(ROOT, "paper_2511_17551_amd", "libdgx.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(dgx_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_2511_17551_amd import build
        build.build()
    return LIB


def test_header_declares_the_boundary():
    names = declared()
    for required in ("dgx_create", "dgx_set_mesh", "dgx_rhs", "dgx_ssprk3_step", "dgx_thermo",
                     "dgx_chem_step", "dgx_check", "dgx_last_error", "dgx_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (dgx_[a-z0-9_]+)$", out, flags=re.M))
    assert set(declared()) <= exported


def test_binding_wraps_every_symbol(lib_path):
    from paper_2511_17551_amd import dgx
    assert set(dgx.EXPORTED) == set(declared())
    for n in declared():
        assert callable(getattr(dgx, n, None)), n


def test_errors_without_a_context(lib_path):
    """Argument checks run before any device work: NULL contexts are rejected."""
    lib = ctypes.CDLL(lib_path)
    lib.dgx_rhs.restype = ctypes.c_int
    lib.dgx_rhs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.dgx_rhs(None, None, 0.0, None, None) < 0
    lib.dgx_create.restype = ctypes.c_int
    lib.dgx_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.dgx_create(None, None) < 0
