"""CPU builds under AddressSanitizer and UndefinedBehaviorSanitizer:

* the FP64 oracle (oracle/gf_oracle.c) with a driver that runs every fill mode
  and the adjoint on seeded tiny problems (oracle/sanitize_check.c);
* the host code of the HIP library (guidefill.hip, sanitizers on the host
  pass) with a driver that goes through every C entry point's validation, workspace
  layout and tile geometry (paper_1611_05319_amd/csrc/abi_check.cpp); every
  call it makes is rejected before a kernel launch.

Both builds use the sanitizers on host code only; no GPU is involved."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
CLANGXX = "/opt/rocm/llvm/bin/clang++"


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fopenmp",
          os.path.join(ROOT, "oracle", "gf_oracle.c"), os.path.join(ROOT, "oracle", "sanitize_check.c"),
          "-o", exe, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="1")
    r = _run([exe], env=env)
    assert "oracle sanitize check ok" in r.stdout


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)), reason="ROCm missing")
def test_library_host_code_under_asan_and_ubsan(tmp_path):
    lib = str(tmp_path / "libgf_sanitized.so")
    src = os.path.join(ROOT, "paper_1611_05319_amd", "csrc")
    inc = os.path.join(ROOT, "include")
    # sanitizers on the host pass only; the device code is built (its objects
    # must be present for the library to load) but never run
    _run([HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-shared",
          "-ffp-contract=off", "-Xarch_host", "-g", "-Xarch_host", "-fno-omit-frame-pointer",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-sanitize-recover=all", f"-I{inc}",
          os.path.join(src, "guidefill.hip"), "-o", lib])
    exe = str(tmp_path / "abi_check")
    _run([CLANGXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all", f"-I{inc}",
          os.path.join(src, "abi_check.cpp"), lib, f"-Wl,-rpath,{tmp_path}", "-o", exe])
    # leaks of the HIP runtime's own start-up are not this library's
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    r = _run([exe], env=env)
    assert "abi sanitize check ok" in r.stdout
