"""Build libgsr.so (HIP for gfx950 + host C++) in-tree.

    python -m paper_2403_11367_amd.build

Compiles every source under csrc/ with hipcc (g++ for the host-only crop),
into paper_2403_11367_amd/_build/, and links paper_2403_11367_amd/libgsr.so.
The geometry kernels (records and depth keys that must match bit for bit)
are built without floating-point contraction and with correctly rounded
float32 division and square root.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libgsr.so")
ARCH = os.environ.get("GSR_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    "-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]
STRICT_FP = ["-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt", "-fno-fast-math"]

SOURCES = [
    ("geometry.hip", "hip", STRICT_FP),
    ("sort.hip", "hip", []),
    ("blend.hip", "hip", []),
    ("backward.hip", "hip", []),
    ("ncc.hip", "hip", []),
    ("scorer.hip", "hip", []),
    ("scorer_rt.cpp", "hip", ["-x", "hip"]),
    ("runtime.cpp", "hip", ["-x", "hip"]),
    ("crop.cpp", "cxx", []),
]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found; install ROCm or set HIPCC")


# Host AddressSanitizer build (libgsr_asan.so, for the CPU tests of the host code):
# the HIP sources instrument their host pass only, and the host-only source is
# built with the same clang so that one ASan runtime serves the library.
ASAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
BUILD_ASAN = os.path.join(PKG, "_build_asan")
LIB_ASAN = os.path.join(PKG, "libgsr_asan.so")


def _clangxx() -> str:
    return os.path.join(os.path.dirname(os.path.realpath(_hipcc())), "..", "lib", "llvm", "bin", "clang++")


def asan_runtime() -> str:
    """Path of the clang ASan runtime that libgsr_asan.so needs preloaded."""
    import glob
    llvm = os.path.realpath(os.path.join(os.path.dirname(os.path.realpath(_hipcc())), "..", "lib", "llvm"))
    hits = sorted(glob.glob(os.path.join(llvm, "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise RuntimeError("clang ASan runtime not found")
    return hits[-1]


def _compile(src: str, kind: str, extra: list, asan: bool = False) -> str:
    obj = os.path.join(BUILD_ASAN if asan else BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if kind == "hip":
        cmd = [_hipcc(), *HIP_FLAGS, *extra, *(ASAN_HOST if asan else []), "-c", path, "-o", obj]
    elif asan:
        cmd = [os.path.realpath(_clangxx()), "-O1", "-g", "-std=c++17", "-fPIC", "-Wall", "-fsanitize=address",
               "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-c", path, "-o", obj]
    else:
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include"),
               "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    noise = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()
             and "warning generated" not in ln and "warnings generated" not in ln]
    if noise:
        sys.stderr.write("\n".join(noise) + "\n")
    return obj


def build(verbose: bool = False, asan: bool = False) -> str:
    """Build libgsr.so, or with asan the host-instrumented libgsr_asan.so."""
    out_dir, lib = (BUILD_ASAN, LIB_ASAN) if asan else (BUILD, LIB)
    os.makedirs(out_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(*s, asan=asan), SOURCES))
    tmp = lib + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, *(ASAN_HOST if asan else []), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True, asan="--asan" in sys.argv)
