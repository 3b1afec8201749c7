"""Build libkdtree.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2210_12859_amd.build

Every source is compiled to an object in ``_build/`` in parallel, then linked
into ``paper_2210_12859_amd/libkdtree.so``.  Floating-point flags keep the
squared distances bit-identical to plain IEEE binary32 arithmetic: no
contraction into FMA, denormals preserved; packed FP32 instructions are
disabled.
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
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libkdtree.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# (source, compiled for the device, extra flags)
SOURCES = [
    ("kd_api.cpp", True, []),
    ("kd_build_host.cpp", False, []),
    ("kd_traverse.hip", True, []),
    ("kd_sort.hip", True, []),
    # matrix-core results in ordinary VGPRs (the MLP kernels read every
    # accumulator back on the vector ALU; no accumulator-register copies)
    ("kd_mlp.hip", True, ["-mllvm", "-amdgpu-mfma-vgpr-form"]),
    ("kd_model.cpp", True, []),
    ("kd_batch.cpp", True, []),
    ("kd_autotune.cpp", True, []),
    ("kd_noalloc.hip", True, []),
    ("kd_build_gpu.hip", True, []),
    ("kd_range_all.hip", True, []),
]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall",
          "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]
DEVICE = ["--offload-arch=gfx950", "-fno-gpu-flush-denormals-to-zero", "-fno-gpu-rdc",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str, is_hip: bool, extra: list) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON]
    if is_hip:
        cmd += ["-x", "hip", *DEVICE, *extra]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip():
        # host-pass warnings about the packed-fp32 feature are expected
        lines = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln]
        if any(ln.strip() for ln in lines):
            sys.stderr.write("\n".join(lines) + "\n")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(*s), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def clean() -> None:
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    build()
