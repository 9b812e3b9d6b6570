"""Compile libdfpt2.so for gfx950 in-tree.

Every HIP translation unit is compiled with hipcc for gfx950 only, packed-FP32
instruction selection disabled, and linked into ``lib/libdfpt2.so`` next to
this file.  ``python -m paper_2312_07008_amd.build`` rebuilds it.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libdfpt2.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = [
    "api.cpp",
    "pair_f64.hip",
    "density_f64.hip",
    "util.hip",
    "eigh.hip",
    "fno.hip",
    "gemm_f64.hip",
    "correction.cpp",
    "naf.cpp",
    "ladder.cpp",
    "active_particle.hip",
    "cumulant.hip",
    "split.hip",
    "pair_bf16_v.hip",
    "pair_fp8.hip",
    "pair_i8.hip",
    "pair_i8_v.hip",
    "split_t.hip",
    "epi_split_bf16.hip",
    "density_bf16.hip",
    "density_i8.hip",
    "active.hip",
    "screen.hip",
    "prof.cpp",
]

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + INCLUDE, "-Wno-unused-result"]


def _compile(src: str, obj: str, verbose: bool) -> None:
    cmd = [HIPCC] + COMMON + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "ignoring feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    if verbose and out.strip():
        print(out, flush=True)


def build(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    objdir = os.path.join(LIBDIR, "obj")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    jobs = min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], verbose), zip(SOURCES, objs)))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
