"""Sanitizer builds on the CPU (no GPU needed): the FP64 oracle and the
library's host runtime under AddressSanitizer and UndefinedBehaviorSanitizer.

* oracle/sanitize_check.c drives every oracle function on small lattices with
  solid sites (gcc -fsanitize=address,undefined, OpenMP on two threads).
* tests/sanitize_host_abi.cpp drives the C ABI's argument and handle checks
  against a copy of liblbm355 whose HOST code is built with the sanitizers
  (-Xarch_host before each flag); device code is built as usual.  With no GPU
  present creation fails cleanly with LB_EHIP; with one, small lattices are
  created, stepped and destroyed.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

pytestmark = pytest.mark.slow

SAN_ENV = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, " ".join(cmd) + "\n" + res.stdout[-4000:] + res.stderr[-4000:]
    return res


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_check")
    _run(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wall", "-Werror", "-o", exe,
          os.path.join(ORACLE, "d3q19_oracle.c"), os.path.join(ORACLE, "d2q9_oracle.c"),
          os.path.join(ORACLE, "sanitize_check.c"), "-lm"])
    res = _run([exe], env=SAN_ENV, timeout=300)
    assert "sanitize_check ok" in res.stdout


def test_host_runtime_under_address_and_undefined_sanitizers(tmp_path):
    from paper_2409_16781_amd import _build

    host_san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"):
        host_san += ["-Xarch_host", f]
    lib = _build.build(out=str(tmp_path / "liblbm355_san.so"), extra=host_san, objdir=str(tmp_path / "obj"))
    exe = str(tmp_path / "sanitize_host_abi")
    clangxx = "/opt/rocm/llvm/bin/clang++"
    _run([clangxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-o", exe,
          os.path.join(ROOT, "tests", "sanitize_host_abi.cpp"), lib, "-Wl,-rpath," + str(tmp_path)])
    res = _run([exe], env=SAN_ENV, timeout=300)
    assert "sanitize_host_abi ok" in res.stdout
