"""Build ``libwx.so`` (the HIP library behind include/wx.h) for gfx950, in-tree.

Usage: ``python -m paper_1802_05839_amd._build`` (or ``__graft_entry__.build()``).
Always recompiles.  hipcc cross-compiles gfx950 device code on a machine
without a GPU.
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
LIB = os.path.join(PKG, "libwx.so")

SOURCES = ["wx_host.hip", "wx_mlp_host.hip", "k_dycore.hip", "k_physics.hip", "k_mlp.hip",
           "k_surrogate.hip", "k_judge.hip", "k_fused.hip", "k_reduced.hip", "k_hevi.hip", "hevi_host.hip", "k_physics_scan.hip"]

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-result",
    "-Wno-pass-failed",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libwx.so)")


def build(verbose: bool = False) -> str:
    objs = []
    out_dir = os.path.join(PKG, "_objs")
    os.makedirs(out_dir, exist_ok=True)
    cc = hipcc()
    for src in SOURCES:
        obj = os.path.join(out_dir, src.replace(".hip", ".o"))
        cmd = [cc, *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
