"""In-tree build of the native libraries.

* libpmgen.so -- seeded input generator (gcc, OpenMP)
* libpm.so    -- the C-ABI pruning library: host engine (C++) and HIP kernels
                 for gfx950, compiled with hipcc.

Objects go to _build/ at the repository root; the shared libraries are
written next to the Python modules that load them.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build")
GEN_LIB = os.path.join(PKG, "inputs", "libpmgen.so")
PM_LIB = os.path.join(PKG, "libpm.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for all device code.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
             "-Wno-unused-command-line-argument",
             f"-I{INCLUDE}", f"-I{CSRC}"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build_gen() -> str:
    src = os.path.join(PKG, "inputs", "gen.c")
    tmp = GEN_LIB + ".tmp"
    _run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", src, "-o", tmp])
    os.replace(tmp, GEN_LIB)
    return GEN_LIB


def _compile_one(src: str) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    if src.endswith(".hip"):
        cmd = [HIPCC, *HIP_FLAGS, "-x", "hip", "-c", src, "-o", obj]
    else:
        # host-only translation units: still compiled by hipcc for the HIP
        # runtime headers, without device code generation
        cmd = [HIPCC, "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
               f"-I{INCLUDE}", f"-I{CSRC}", "-D__HIP_PLATFORM_AMD__", "-c", src, "-o", obj]
    _run(cmd)
    return obj


def build_pm(jobs: int = 8) -> str:
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    if not srcs:
        raise RuntimeError("no library sources found")
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        objs = list(ex.map(_compile_one, srcs))
    tmp = PM_LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    os.replace(tmp, PM_LIB)
    return PM_LIB


def build_all() -> None:
    build_gen()
    build_pm()


def clean() -> None:
    shutil.rmtree(OBJDIR, ignore_errors=True)
