"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the code that
runs on the CPU only: the oracle and certificate sources (oracle/) and the
host-side level-range choice of the batched search (csrc/level_cover.h).
Each is built into a driver of its own with gcc/g++ and run on many seeded
inputs; any out-of-bounds access, integer overflow or leak fails the run.
(The HIP library itself has no sanitizer build: GPU sanitizers are not
available here.)"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests")
FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
         "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd_build, exe):
    subprocess.run(cmd_build, check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    exe = str(tmp_path / "sanitize_oracle")
    out = _run(["gcc", "-std=c11", *FLAGS, "-o", exe, os.path.join(HERE, "sanitize_oracle.c"),
                os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "oracle", "certify.c")], exe)
    assert "0 failures" in out


def test_level_cover_under_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ is not available")
    exe = str(tmp_path / "sanitize_level_cover")
    out = _run(["g++", "-std=c++17", *FLAGS, "-o", exe, os.path.join(HERE, "sanitize_level_cover.cpp")],
               exe)
    assert "0 bad" in out
