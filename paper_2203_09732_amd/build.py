"""Builds libmbl.so for gfx950 with hipcc, in-tree.

    python paper_2203_09732_amd/build.py        (or build() from Python)

Each .hip translation unit under csrc/ is compiled in parallel and linked
into paper_2203_09732_amd/libmbl.so; then the C example program
(examples/mbl_example.c, a plain C99 caller of the C ABI) is compiled with
the host C compiler into paper_2203_09732_amd/mbl_example. It always
recompiles.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmbl.so")
EXAMPLE = os.path.join(HERE, "mbl_example")
CC = os.environ.get("CC", "gcc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]

SOURCES = ["kernels.hip", "minres.hip", "lanczos.hip", "batched.hip", "adjoint.hip", "schmidt.hip",
           "noalloc.hip", "wgsolve.hip", "api.hip"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(6, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    cmd = [CC, "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(HERE, "examples", "mbl_example.c"), "-o", EXAMPLE,
           "-L", HERE, "-lmbl", "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"C example build failed:\n{r.stderr}")
    if verbose:
        print("built", OUT, "and", EXAMPLE)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
