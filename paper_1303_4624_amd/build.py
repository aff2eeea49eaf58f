"""Build liblbm.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc.

    python -m paper_1303_4624_amd.build          # or build_library() from Python

The library is written next to this file.  Every HIP translation unit is
compiled for gfx950 only, with packed-FP32 instruction generation disabled.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(HERE, "liblbm.so")
# One translation unit per model (and per precision for D3Q95), so that the
# heavy kernel instantiations compile in parallel.
SOURCES = ["lbm_kernels_d3q95_f32s.hip", "lbm_kernels_d3q95_f64.hip", "lbm_kernels_d2q33.hip",
           "lbm_kernels_lower.hip", "lbm_kernels_common.hip", "lbm_api.cpp",
           "lbm_model_host.cpp"]
# Host-only sources compiled by the host C++ compiler (binary128 arithmetic).
HOST_SOURCES = {"lbm_model_host.cpp"}
ARCH = "gfx950"

# -ffp-contract=off: no multiply-add is fused unless the source says fma(),
# so every kernel that computes a quantity rounds it the same way (the
# two-buffer and in-place updates agree bit for bit by construction).
COMMON = [
    "-O3", "-std=c++20", "-fPIC", "-fvisibility=hidden", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, obj: str) -> None:
    if src in HOST_SOURCES:
        cxx = shutil.which("g++") or "g++"
        cmd = [cxx, "-O2", "-std=c++20", "-fPIC", "-fvisibility=hidden", "-I", INCLUDE,
               "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
    else:
        cmd = [_hipcc(), "-x", "hip", f"--offload-arch={ARCH}", *COMMON, "-c",
               os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")


def build_library(verbose: bool = True) -> str:
    """Compile every source and link liblbm.so; returns its path."""
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    objs = [os.path.join(build_dir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(lambda so: _compile(*so), zip(SOURCES, objs)))
    tmp = LIB_PATH + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           "-lquadmath"]
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout)
    os.replace(tmp, LIB_PATH)
    if verbose:
        print(f"built {LIB_PATH}")
    return LIB_PATH


if __name__ == "__main__":
    build_library()
    sys.exit(0)
