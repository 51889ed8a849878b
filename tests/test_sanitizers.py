"""CPU runs under AddressSanitizer and UndefinedBehaviorSanitizer.

* The oracle (plain C) with a driver that exercises every oracle entry point
  on small inputs with known results (tests/sanitize/oracle_driver.c).
* The host side of the HIP library, built with host sanitizers, with a
  driver that calls every C-ABI entry point with arguments its validation
  must refuse (tests/sanitize/abi_driver.c); no call reaches a device, so
  this runs without a GPU.
A sanitizer report makes the driver exit non-zero.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
OUT = os.path.join(HERE, "_build")
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers():
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_driver")
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp", "-std=c11",
          os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "oracle_driver.c"),
          "-lm", "-o", exe])
    r = _run([exe], env=dict(SAN_ENV, ASAN_OPTIONS="detect_leaks=1"))
    assert "all checks held" in r.stdout


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not available")
def test_abi_validation_under_sanitizers():
    from paper_1012_2273_amd import build
    os.makedirs(OUT, exist_ok=True)
    lib = build.build(sanitize=True)            # host sanitizers, rebuilt only when stale
    exe = os.path.join(OUT, "abi_driver")
    libdir = os.path.dirname(lib)
    _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
          os.path.join(HERE, "abi_driver.c"), "-o", exe, "-L", libdir,
          "-l:" + os.path.basename(lib), "-Wl,-rpath," + libdir])
    r = _run([exe], env=SAN_ENV)
    assert "all checks held" in r.stdout
