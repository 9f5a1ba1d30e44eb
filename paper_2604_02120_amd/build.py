"""Build libgsblend.so (HIP, gfx950 only) in-tree with hipcc.

    python -m paper_2604_02120_amd.build

Each translation unit is compiled to an object in ``_build/`` (in parallel), then linked into
``paper_2604_02120_amd/libgsblend.so``. Builds always recompile.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libgsblend.so")
SOURCES = ["capi.hip", "bin.hip", "blend.hip", "project.hip"]
# the attainable-rate microbenchmark (bench.py --peaks): a library of its own, not part of the ABI
PEAKS_LIB = os.path.join(PKG, "libgsbpeaks.so")
PEAKS_SRC = "peaks.hip"
# per-file extras: the blend kernels never produce NaN from in-contract inputs (-inf is used, NaN
# never), so min/max need no NaN canonicalisation
EXTRA = {"blend.hip": ["-fno-honor-nans"]}

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-munsafe-fp-atomics",
    # keep per-lane atomics as single instructions (no readlane loop around them)
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    # packed FP32 (v_pk_*_f32) stays off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *EXTRA.get(src, []), "-I", os.path.join(PKG, "..", "include"), "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def _link(objs, lib: str) -> None:
    tmp = lib + f".tmp{os.getpid()}"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES) + 1, 8)) as ex:
        objs = list(ex.map(_compile, SOURCES + [PEAKS_SRC]))
    _link(objs[:-1], LIB)
    _link(objs[-1:], PEAKS_LIB)
    if verbose:
        print(f"built {LIB} and {PEAKS_LIB}")
    return LIB


def clean() -> None:
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    build(verbose=True)
