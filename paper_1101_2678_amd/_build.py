"""Builds libaco.so (the HIP kernels and the C ABI) in-tree for gfx950.

Flags that matter for the arithmetic:
  -ffp-contract=off                 no fused multiply-add unless written
  -fno-gpu-flush-denormals-to-zero  binary32 subnormals are kept
  -fno-fast-math (default)          IEEE division, no reassociation
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                    no packed FP32 instructions
The library links against the HIP runtime that torch loads (same file, via
an rpath), so streams and device pointers handed over by torch belong to the
runtime the kernels are launched on.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB_PATH = os.path.join(PKG, "libaco.so")
SOURCES = ["construct.hip", "construct_split.hip", "construct_nn.hip", "construct_product.hip", "update.hip", "probe.hip", "aco_abi.hip", "batch.hip", "server.hip", "noalloc.hip"]
ARCH = os.environ.get("ACO_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++20",
    "-fPIC",
    "-ffp-contract=off",
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    f"-I{INCLUDE}",
    f"-I{CSRC}",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _torch_lib_dir() -> str | None:
    try:
        import importlib.util

        spec = importlib.util.find_spec("torch")
        if spec is None or spec.origin is None:
            return None
        d = os.path.join(os.path.dirname(spec.origin), "lib")
        return d if os.path.exists(os.path.join(d, "libamdhip64.so")) else None
    except Exception:
        return None


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    os.makedirs(BUILD_DIR, exist_ok=True)
    hipcc = _hipcc()
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, src.replace(".hip", ".o"))
        cmd = [hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB_PATH + ".tmp"
    torch_lib = _torch_lib_dir()
    if torch_lib:
        link = ["g++", "-shared", "-o", tmp, *objs, os.path.join(torch_lib, "libamdhip64.so"),
                f"-Wl,-rpath,{torch_lib}"]
    else:
        link = [hipcc, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(link), file=sys.stderr)
    subprocess.run(link, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(force=True, verbose=True))
