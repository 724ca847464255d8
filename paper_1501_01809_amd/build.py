"""Build the HIP library ``libfem.so`` for gfx950 (hipcc, no JIT, in-tree).

Steps: regenerate ``csrc/fem_tables.h`` from the exact reference integrals,
compile every source for ``--offload-arch=gfx950`` with packed-FP32
instruction selection disabled, link a shared library next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfem.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = ["fem_api.cpp", "fem_sparsity.hip", "fem_assemble.hip", "fem_nl.hip", "fem_elast.hip", "fem_serve.cpp", "fem_global.hip", "fem_bc.hip", "fem_facet.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_tables.py"),
                           os.path.join(CSRC, "fem_tables.h")],
                          stdout=subprocess.DEVNULL)
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_elast_tables.py"),
                           os.path.join(CSRC, "fem_elast_tables.h")],
                          stdout=subprocess.DEVNULL)
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_facet_tables.py"),
                           os.path.join(CSRC, "fem_facet_tables.h")],
                          stdout=subprocess.DEVNULL)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
