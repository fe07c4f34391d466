"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code.

* The FP64 oracle, compiled whole with gcc and both sanitizers, runs every
  entry point (Philox, axes, fields, energy, single and batched runs with the
  OpenMP paths, loop statistics, the adjoint, the Newell tensor) on ragged
  grids with and without magnetostatics; leaks are errors.
* The library's host code, compiled by hipcc with the sanitizers on the host
  pass only (device code has none), runs everything that needs no GPU: the
  validation of every argument, the level compiler and workspace layout of
  the benchmark's workloads, and the error paths of sllg_init.  This build
  found a use of the context after its release in the path that refuses a
  workspace that is too small.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"

ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    return r.returncode, r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    rc, out = run(["gcc", "-g", "-O1", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
                   "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-Wall",
                   "-o", exe, os.path.join(HERE, "sanitize", "oracle_driver.c"), "-lm"])
    assert rc == 0, out
    rc, out = run([exe], env=dict(ENV, OMP_NUM_THREADS="2"), timeout=600)
    assert rc == 0 and "all calls clean" in out, out


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not found")
def test_library_host_code_under_address_and_undefined_sanitizers(tmp_path):
    lib = str(tmp_path / "libsllg_asan.so")
    # sanitizers on the host pass only; device code unoptimised (it only has
    # to link: no kernel runs here)
    rc, out = run([HIPCC, "--offload-arch=gfx950", "-g", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                   "-Xarch_host", "-O1", "-Xarch_device", "-O0",
                   "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                   "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                   "-o", lib, os.path.join(ROOT, "paper_1912_00310_amd", "csrc", "sllg_host.hip")], timeout=900)
    assert rc == 0, out
    exe = str(tmp_path / "host_driver")
    rc, out = run([CLANG, "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                   "-fno-omit-frame-pointer", "-o", exe, os.path.join(HERE, "sanitize", "host_driver.c"), lib,
                   "-Wl,-rpath," + str(tmp_path)])
    assert rc == 0, out
    rc, out = run([exe], env=ENV, timeout=300)
    assert rc == 0 and "all calls clean" in out, out
