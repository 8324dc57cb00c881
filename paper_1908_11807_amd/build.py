"""Build libabx.so (HIP, gfx950) in-tree with hipcc.

Usage: ``python -m paper_1908_11807_amd.build`` or ``build_library()``.
Every HIP source under ``csrc/`` is compiled to an object in
``_build/`` (in parallel) and linked into ``paper_1908_11807_amd/libabx.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libabx.so")
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libabx)")


def common_flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        "-ffp-contract=off",                       # no implicit fused multiply-add
        "-fhip-fp32-correctly-rounded-divide-sqrt",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
        f"-I{INCLUDE}", f"-I{CSRC}",
    ]


# ThreadSanitizer instruments the host code only (the scheduler and the ABI);
# device code is built as usual
TSAN_FLAGS = ["-Xarch_host", "-fsanitize=thread", "-g"]


def _compile(src: str, out_dir: str = BUILD_DIR, extra=()) -> str:
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = [hipcc(), *common_flags(), *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build_library(verbose: bool = True) -> str:
    """Compile every HIP source for gfx950 and link libabx.so (always rebuilds)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def tsan_runtime() -> str:
    """The ThreadSanitizer runtime of the ROCm clang (preloaded into the
    process that loads the sanitised library)."""
    import glob as _g
    for c in sorted(_g.glob("/opt/rocm*/lib/llvm/lib/clang/*/lib/linux/libclang_rt.tsan-x86_64.so")):
        return c
    raise RuntimeError("no ThreadSanitizer runtime found under /opt/rocm")


def build_tsan_library() -> str:
    """libabx with its host code built under ThreadSanitizer, in _build/tsan
    (for the CPU tests of the serving scheduler; never shipped)."""
    out_dir = os.path.join(BUILD_DIR, "tsan")
    os.makedirs(out_dir, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda src: _compile(src, out_dir, TSAN_FLAGS), srcs))
    lib = os.path.join(out_dir, "libabx_tsan.so")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=thread",
           "-o", lib, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    return lib


if __name__ == "__main__":
    build_library()
    sys.exit(0)
