"""Build libjkcals.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

Usage: ``python -m paper_2112_03985_amd.build`` or ``build()`` from Python.
Objects go to ``_build/`` at the repository root; the shared library lands
next to this file so the binding finds it in-tree.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libjkcals.so")
LIB_ASAN = os.path.join(PKG, "libjkcals_asan.so")

SOURCES = ["api.cpp", "prep.hip", "update.hip", "mttkrp_f64.hip", "mttkrp_split.hip", "postprocess.hip", "tree.hip", "allmode.hip", "mttkrp_narrow.hip"]

ARCH = "gfx950"
# -packed-fp32-ops: keep the compiler from forming packed float32 ops.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-Wall",
          "-Wno-unused-result", "-I" + os.path.join(ROOT, "include")]


def _hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"]
    cmd = [_hipcc()] + lang + COMMON + DEVICE_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def _link(objs, out: str) -> None:
    tmp = out + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, out)


def build_host_asan(objs) -> str:
    """The host-sanitizer build: the C ABI's validation, planning and launch
    code (api.cpp) compiled with AddressSanitizer on its host side only
    (each -fsanitize= behind -Xarch_host; the GPU code is the normal build),
    linked with the other objects into libjkcals_asan.so.  Load it with the
    clang ASan runtime preloaded and JKCALS_LIBRARY pointing at it
    (tests/test_host_asan.py)."""
    os.makedirs(os.path.join(BUILD, "asan"), exist_ok=True)
    src = "api.cpp"
    obj = os.path.join(BUILD, "asan", "api.o")
    cmd = ([_hipcc(), "-x", "hip", "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
            "-Wall", "-Wno-unused-result", "-I" + os.path.join(ROOT, "include")] + DEVICE_FLAGS +
           ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
            "-c", os.path.join(CSRC, src), "-o", obj])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s (sanitizer build):\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    _link([obj] + [o for o in objs if os.path.basename(o) != "api.o"], LIB_ASAN)
    return LIB_ASAN


def build(verbose: bool = False) -> str:
    """Compile every source (always; no staleness shortcuts) and link; then
    the host-sanitizer variant of the library."""
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    _link(objs, LIB)
    build_host_asan(objs)
    if verbose:
        print("built", LIB, "and", LIB_ASAN)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
