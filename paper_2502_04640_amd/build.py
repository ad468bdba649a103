"""Compile libxm.so (HIP, gfx950) in place next to this file.

    python -m paper_2502_04640_amd.build        # or build() from Python

Each source is compiled to an object with hipcc, then linked into a shared
library; the objects live in _build/ (not part of the sources).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libxm.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["sort.hip", "build_q.hip", "spmm.hip", "manifold.hip", "certify.hip", "solver.hip",
           "round.hip", "adjoint.hip", "noalloc.hip", "pool.cpp", "api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-I" + os.path.join(ROOT, "include")]


def _compile(src: str, build_dir: str = BUILD, defines=()) -> str:
    obj = os.path.join(build_dir, src + ".o")
    extra = ["-D" + d for d in defines]
    cmd = [HIPCC] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip"] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, out: str = OUT, build_dir: str = BUILD, defines=()) -> str:
    """Compile every source and link `out`.  `defines` (NAME=VALUE strings)
    override the compile-time launch constants of the kernels."""
    os.makedirs(build_dir, exist_ok=True)
    workers = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8"))))
    with ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir, defines), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


# Host-code sanitizer build (AddressSanitizer + UndefinedBehaviorSanitizer on
# the host side of every source; device code as usual), and the driver that
# runs every entry point of the C ABI under it (tests/sanitize/host_driver.cpp).
HOSTSAN_CC = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
HOSTSAN_LD = ["-fsanitize=address", "-fsanitize=undefined", "-fno-gpu-sanitize"]
HOSTSAN_LIB = os.path.join(HERE, "libxm_hostsan.so")
HOSTSAN_DRIVER = os.path.join(ROOT, "tests", "sanitize", "xm_hostsan_driver")


def build_hostsan(verbose: bool = False) -> str:
    bdir = os.path.join(BUILD, "hostsan")
    os.makedirs(bdir, exist_ok=True)

    def cc(src_path, obj):
        cmd = [HIPCC, "-x", "hip"] + FLAGS + HOSTSAN_CC + ["-c", src_path, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src_path}:\n{r.stdout}\n{r.stderr}")
        return obj

    workers = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8"))))
    with ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(lambda s: cc(os.path.join(CSRC, s), os.path.join(bdir, s + ".o")), SOURCES))
    link = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950"] + HOSTSAN_LD + ["-o", HOSTSAN_LIB] + objs
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    drv = cc(os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), os.path.join(bdir, "host_driver.o"))
    exe = [HIPCC, "--offload-arch=gfx950"] + HOSTSAN_LD + ["-o", HOSTSAN_DRIVER, drv, "-L" + HERE, "-lxm_hostsan",
                                                         "-Wl,-rpath,$ORIGIN/../../paper_2502_04640_amd"]
    r = subprocess.run(exe, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"driver link failed:\n{r.stdout}\n{r.stderr}")
    if verbose:
        print("built", HOSTSAN_LIB, "and", HOSTSAN_DRIVER)
    return HOSTSAN_DRIVER


if __name__ == "__main__":
    build(verbose=True)
    if "--hostsan" in sys.argv:
        build_hostsan(verbose=True)
    sys.exit(0)
