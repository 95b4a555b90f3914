"""CPU-side checks of the C-ABI library: it is built, loads, and exports
every entry point declared in include/smf.h (no compute calls here)."""
import ctypes
import os
import re

import pytest

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
    assert not lib.smf_create(1 << 15, 1 << 15, 1, 0)   # 2^30 nodes
    assert b"2^30 - 2" in lib.smf_last_error()
    lib.smf_solve.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.smf_solve(None, None, None) == -1


def test_batch_arg_errors_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.smf_last_error.restype = ctypes.c_char_p
    lib.smf_batch_create.restype = ctypes.c_void_p
    arr = lambda *v: (ctypes.c_int32 * len(v))(*v)
    assert not lib.smf_batch_create(0, arr(1), arr(1), arr(1), arr(0))
    assert b"n >= 1" in lib.smf_last_error()
    assert not lib.smf_batch_create(2, arr(4, 4), arr(4, 0), arr(8, 8), arr(1, 1))
    assert b"volume 1" in lib.smf_last_error()
    assert not lib.smf_batch_create(2, arr(4, 4), arr(4, 4), arr(8, 8), arr(1, -1))
    assert b"volume 1" in lib.smf_last_error()
    # three volumes of 32767^2 columns each: every volume fits, the batch does not
    big = 32767
    assert not lib.smf_batch_create(3, arr(big, big, big), arr(big, big, big), arr(1, 1, 1),
                                    arr(0, 0, 0))
    assert b"2^31 - 1 columns" in lib.smf_last_error()
    for name in ("smf_batch_solve", "smf_batch_flow_values", "smf_batch_energies",
                 "smf_batch_surfaces", "smf_batch_set_param", "smf_batch_get_stat"):
        fn = getattr(lib, name)
        fn.restype = ctypes.c_int
        fn.argtypes = [ctypes.c_void_p] * (4 if name == "smf_batch_solve" else
                                           3 if name in ("smf_batch_surfaces", "smf_batch_set_param",
                                                         "smf_batch_get_stat") else 2)
        assert fn(*([None] * len(fn.argtypes))) == -1, name


def test_python_binding_lists_header_symbols():
    src = open(os.path.join(ROOT, "paper_2601_17026_amd", "smf.py")).read()
    for n in declared():
        assert n in src, n


def test_tune_cache_roundtrip_without_gpu(tmp_path):
    # the autotuner's cache: classes keyed by (ceil log2 K, min(delta, 4),
    # floor log2 columns, soft term); files of five fields per line (no soft
    # flag) still load; load, lookup, save and clear need no device
    lib = ctypes.CDLL(LIB)
    lib.smf_tune_lookup.argtypes = [ctypes.c_int32] * 4 + [ctypes.POINTER(ctypes.c_int64)]
    lib.smf_tune_cache_load.argtypes = [ctypes.c_char_p]
    lib.smf_tune_cache_save.argtypes = [ctypes.c_char_p]
    lib.smf_last_error.restype = ctypes.c_char_p

    def look(nx, ny, K, d):
        out = ctypes.c_int64(-1)
        assert lib.smf_tune_lookup(nx, ny, K, d, ctypes.byref(out)) == 0
        return out.value

    assert lib.smf_tune_cache_clear() == 0
    assert look(128, 128, 100, 2) == 0
    src = tmp_path / "tune.txt"
    src.write_text("7 2 14 8 12345\n9 4 18 3 999\n")
    assert lib.smf_tune_cache_load(str(src).encode()) == 0
    assert look(128, 128, 100, 2) == 8      # K 100 -> 7 bits, 16384 columns -> 14
    assert look(128, 128, 128, 2) == 8
    assert look(128, 128, 129, 2) == 0      # K 129 -> 8 bits
    assert look(128, 255, 100, 2) == 8      # 32640 columns -> 14
    assert look(128, 256, 100, 2) == 0      # 32768 columns -> 15
    assert look(512, 512, 384, 7) == 3      # delta above 4 shares the class of 4
    # a class with the soft smoothness term (sixth field layout) is separate
    soft = tmp_path / "soft.txt"
    soft.write_text("7 2 14 1 4 777\n")
    assert lib.smf_tune_cache_load(str(soft).encode()) == 0
    assert look(128, 128, 100, 2) == 8
    dst = tmp_path / "out.txt"
    assert lib.smf_tune_cache_save(str(dst).encode()) == 0
    assert sorted(dst.read_text().split("\n")) == sorted(
        ["", "7 2 14 0 8 1 12345", "7 2 14 1 4 1 777", "9 4 18 0 3 1 999"])
    assert lib.smf_tune_cache_load(str(tmp_path / "missing.txt").encode()) == -1
    assert b"cannot open" in lib.smf_last_error()
    out = ctypes.c_int64()
    assert lib.smf_tune_lookup(0, 1, 1, 0, ctypes.byref(out)) == -1
    assert lib.smf_tune_cache_clear() == 0
    assert look(128, 128, 100, 2) == 0


def test_tune_cache_env_file_without_gpu(tmp_path):
    # SMF_TUNE_CACHE names a cache file that is read on first use
    import subprocess
    import sys
    src = tmp_path / "tune.txt"
    src.write_text("6 1 10 12 777\n")
    code = ("import ctypes; lib = ctypes.CDLL(%r); out = ctypes.c_int64();"
            "lib.smf_tune_lookup.argtypes = [ctypes.c_int32] * 4 + [ctypes.POINTER(ctypes.c_int64)];"
            "assert lib.smf_tune_lookup(32, 32, 64, 1, ctypes.byref(out)) == 0;"
            "print(out.value)") % LIB
    env = dict(os.environ, SMF_TUNE_CACHE=str(src))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    assert r.stdout.strip() == "12"


def test_no_gpu_fails_loudly():
    # with no GPU, creating a solver raises and names the missing device:
    # nothing on the product path falls back to the CPU
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2601_17026_amd import smf
    for make in (lambda: smf.Solver(4, 4, 4, 1), lambda: smf.BatchSolver([(4, 4, 4, 1), (3, 5, 6, 0)])):
        with pytest.raises(smf.SmfError) as ei:
            make()
        assert "no usable HIP device" in str(ei.value)


def test_device_memory_budget_refuses_before_allocating(monkeypatch):
    # SMF_DEVICE_MEM_LIMIT below what a handle needs: SMF_ERR_NOMEM from
    # smf_create, decided before any device call (so also without a GPU)
    from paper_2601_17026_amd import smf
    monkeypatch.setenv("SMF_DEVICE_MEM_LIMIT", "1000000")   # 1 MB; 64x64x64 needs ~8.6 MB
    for make in (lambda: smf.Solver(64, 64, 64, 1), lambda: smf.BatchSolver([(64, 64, 64, 1)] * 2)):
        with pytest.raises(smf.SmfError) as ei:
            make()
        assert "SMF_DEVICE_MEM_LIMIT" in str(ei.value)
    lib = smf._lib
    assert lib.smf_create(64, 64, 64, 1) is None
    assert b"more than SMF_DEVICE_MEM_LIMIT" in lib.smf_last_error()


def test_every_parameter_key_is_documented():
    # every key smf_set_param accepts is described in the header
    host = open(os.path.join(ROOT, "paper_2601_17026_amd", "csrc", "smf_host.hip")).read()
    body = host[host.index('extern "C" int smf_set_param('):host.index('extern "C" int smf_batch_set_param(')]
    keys = set(re.findall(r'strcmp\(key, "([a-z_]+)"\)', body))
    assert {"relabel_period", "push_phases", "search_quorum", "block_search"} <= keys
    text = open(HEADER).read()
    assert not [k for k in sorted(keys) if f'"{k}"' not in text]
