"""CPU-side checks of the C-ABI library: it is built, loads, and exports
every entry point declared in include/smf.h (no compute calls here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smf.h")
LIB = os.path.join(ROOT, "paper_2601_17026_amd", "_libsmf.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(smf_[a-z_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("smf_create", "smf_solve", "smf_flow_value", "smf_surface", "smf_destroy"):
        assert n in names


def test_library_exports_all_declared_symbols():
    assert os.path.exists(LIB), "library not built"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_arg_errors_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.smf_status_string.restype = ctypes.c_char_p
    lib.smf_last_error.restype = ctypes.c_char_p
    assert lib.smf_status_string(0) == b"ok"
    assert lib.smf_status_string(-4).startswith(b"not converged")
    lib.smf_create.restype = ctypes.c_void_p
    # argument checks happen before any device call
    assert not lib.smf_create(0, 1, 1, 0)
    assert b"nx, ny, K" in lib.smf_last_error()
    assert not lib.smf_create(1 << 16, 1 << 16, 2, 0)
    assert b"2^31" in lib.smf_last_error()
    lib.smf_solve.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.smf_solve(None, None, None) == -1


def test_python_binding_lists_header_symbols():
    src = open(os.path.join(ROOT, "paper_2601_17026_amd", "smf.py")).read()
    for n in declared():
        assert n in src, n
