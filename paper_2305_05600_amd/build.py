"""Builds libhvpic.so (HIP, gfx950) in-tree with hipcc.

All sources under csrc/ go into one shared library exporting the C-ABI of
include/hvpic.h.  Packed FP32 instructions are disabled for the device code.
"""
from __future__ import annotations

import os
import pathlib
import subprocess

PKG = pathlib.Path(__file__).resolve().parent
ROOT = PKG.parent
SOURCES = ["abi.hip", "particles.hip", "sort.hip", "fields.hip", "fields_ext.hip", "ensemble.hip",
           "surrogate.hip", "open.hip"]
LIB = PKG / "libhvpic.so"


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return str(pathlib.Path(rocm) / "bin" / "hipcc")


def build(verbose: bool = False, extra: list[str] | None = None) -> pathlib.Path:
    tmp = PKG / "libhvpic.so.tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
           f"-I{ROOT / 'include'}", f"-I{PKG / 'csrc'}",
           *[str(PKG / "csrc" / s) for s in SOURCES],
           *(extra or []), "-o", str(tmp)]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    tmp.replace(LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
