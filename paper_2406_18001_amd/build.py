"""Build the kdcd HIP library for gfx950 in-tree.

Every ``csrc/*.hip`` and ``csrc/*.cpp`` file is compiled with hipcc into
``_build/`` (objects, in parallel) and linked into
``paper_2406_18001_amd/libkdcd.so``.  Packed-FP32 instructions are disabled
for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libkdcd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr}")
    # hipcc's host pass does not know the packed-fp32 target feature; that warning is harmless
    noise = [ln for ln in res.stderr.splitlines() if ln.strip() and "packed-fp32-ops" not in ln
             and "not a recognized feature" not in ln]
    if noise:
        sys.stderr.write("\n".join(noise) + "\n")
    return obj


PEAK_SRC = os.path.join(PKG, "peak", "peak.hip")
PEAK_LIB = os.path.join(PKG, "libkdcd_peak.so")


def build_peak() -> str:
    """The MFMA / HBM peak microbenchmarks (a library of their own)."""
    tmp = PEAK_LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-shared", PEAK_SRC, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {PEAK_SRC}:\n{res.stderr}")
    os.replace(tmp, PEAK_LIB)
    return PEAK_LIB


def build_library(jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(8, len(srcs))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


ASAN_DIR = os.path.join(BUILD, "asan")
ASAN_RUNTIME = "libclang_rt.asan-x86_64.so"


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime that the host code below links against."""
    found = sorted(glob.glob(os.path.join(os.path.dirname(HIPCC), "..", "llvm", "lib", "clang", "*",
                                          "lib", "linux", ASAN_RUNTIME)))
    if not found:
        raise RuntimeError("clang AddressSanitizer runtime not found")
    return os.path.realpath(found[-1])


def build_asan() -> tuple[str, str]:
    """CPU-side AddressSanitizer build: the library's host code (device code
    is compiled as usual) and the C oracle, both with clang's runtime, into
    _build/asan/.  Run the CPU suite against them with

      LD_PRELOAD=<asan_runtime()> ASAN_OPTIONS=detect_leaks=0 \
      KDCD_LIBRARY=_build/asan/libkdcd.so KDCD_ORACLE_LIBRARY=_build/asan/liboracle.so \
      python -m pytest tests -m "not gpu"
    """
    os.makedirs(ASAN_DIR, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xarch_host", "-g"]

    def comp(src):
        obj = os.path.join(ASAN_DIR, os.path.basename(src) + ".o")
        res = subprocess.run([HIPCC, *FLAGS, *san, "-c", src, "-o", obj], capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc (asan) failed for {src}:\n{res.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(comp, sources()))
    lib = os.path.join(ASAN_DIR, "libkdcd.so")
    res = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-fsanitize=address",
                          "-shared-libasan", *objs, "-o", lib], capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"asan link failed:\n{res.stderr}")
    clang = os.path.join(os.path.dirname(HIPCC), "..", "llvm", "bin", "clang")
    orc = os.path.join(ASAN_DIR, "liboracle.so")
    res = subprocess.run([clang, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                          "-fno-fast-math", "-fopenmp", "-fsanitize=address,undefined",
                          "-fno-sanitize-recover=undefined", "-shared-libasan", "-fPIC", "-shared",
                          os.path.join(ROOT, "oracle", "kdcd_oracle.c"), "-o", orc, "-lm"],
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"oracle asan build failed:\n{res.stderr}")
    return lib, orc


if __name__ == "__main__":
    if "--asan" in sys.argv:
        print(*build_asan(), asan_runtime())
    else:
        print(build_library())
        print(build_peak())
