"""Build libgemm_mi355x.so for gfx950 with hipcc (in-tree, no JIT cache).

    python -m paper_1012_2273_amd.build [--force] [-j N]

Each translation unit under csrc/ is compiled to an object in _build/ (in
parallel), then linked into paper_1012_2273_amd/libgemm_mi355x.so. Objects are
rebuilt when the unit or any header under csrc/ or include/ is newer.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libgemm_mi355x.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++20", "-fPIC",
    # keep the compiler from forming packed binary32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function",
    # MFMA accumulators in architectural VGPRs: on gfx950 a binary64 MFMA that
    # writes AccVGPRs issues at about half rate (measured: ~138 vs 64 cycles
    # per v_mfma_f64_16x16x4 per wave)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
]


def _sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _headers():
    return glob.glob(os.path.join(CSRC, "*.h*")) + glob.glob(os.path.join(INCLUDE, "*.h"))


def _stale(target, deps):
    if not os.path.exists(target):
        return True
    t = os.path.getmtime(target)
    return any(os.path.getmtime(d) > t for d in deps)


def _compile(src, force, build_dir=BUILD, extra=()):
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    if force or _stale(obj, [src, *_headers(), os.path.abspath(__file__)]):
        cmd = [HIPCC, *CFLAGS, *extra, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer for the CPU checks
# of the ABI's validation paths (the device code is built as usual).
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def build(force: bool = False, jobs: int | None = None, sanitize: bool = False,
          out: str | None = None) -> str:
    """Compile every unit under csrc/ and link the library. ``sanitize`` adds
    the host sanitizers (objects under _build/san/, library at ``out``)."""
    build_dir = os.path.join(BUILD, "san") if sanitize else BUILD
    lib = out or (os.path.join(build_dir, "libgemm_mi355x_san.so") if sanitize else LIB)
    os.makedirs(build_dir, exist_ok=True)
    srcs = _sources()
    jobs = jobs or min(8, os.cpu_count() or 1)
    extra = SAN_FLAGS if sanitize else []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force, build_dir, extra), srcs))
    if force or _stale(lib, objs):
        tmp = lib + ".tmp%d" % os.getpid()
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, *extra]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stderr}")
        os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--force", action="store_true")
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("--sanitize", action="store_true",
                    help="host AddressSanitizer/UBSan build under _build/san/ (CPU checks)")
    a = ap.parse_args()
    print(build(a.force, a.j, sanitize=a.sanitize))
    sys.exit(0)
