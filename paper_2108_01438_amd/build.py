"""Build liboct.so (HIP for gfx950) in-tree with hipcc.

Usage: python paper_2108_01438_amd/build.py   (run as a script: importing the
package would load the previously built library)
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "liboct.so")
SOURCES = ["oct_lateral.hip", "oct_nufft.hip", "oct_prox.hip", "oct_direct.hip", "oct_literal.hip", "oct_dtcwt.hip", "oct_api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled: plain float code is compiled to
# scalar-per-lane FP32 only.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build_library(verbose: bool = True) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


# Host sanitizer build: the library's sources and tests/sanitize/host_sanitize_driver.cpp
# linked into one executable whose HOST code carries AddressSanitizer and
# UndefinedBehaviorSanitizer (each -fsanitize= follows -Xarch_host: the device
# code is built as usual).  tests/test_gpu_host_sanitizers.py runs it.
SAN_DIR = os.path.join(BUILD_DIR, "sanitize")
SAN_DRIVER = os.path.join(ROOT, "tests", "sanitize", "host_sanitize_driver.cpp")
SAN_EXE = os.path.join(ROOT, "tests", "sanitize", "host_sanitize_driver")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-g1"]


def _compile_san(path: str) -> str:
    obj = os.path.join(SAN_DIR, os.path.basename(path) + ".o")
    cmd = [HIPCC] + FLAGS + SAN_FLAGS + ["-x", "hip", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {path}:\n{r.stdout}\n{r.stderr}")
    return obj


def build_sanitize_driver(verbose: bool = True) -> str:
    os.makedirs(SAN_DIR, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES] + [SAN_DRIVER]
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(_compile_san, srcs))
    tmp = SAN_EXE + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950"] + SAN_FLAGS + ["-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, SAN_EXE)
    if verbose:
        print(f"built {SAN_EXE}")
    return SAN_EXE


if __name__ == "__main__":
    build_library()
    if "--sanitize" in sys.argv:
        build_sanitize_driver()
    sys.exit(0)
