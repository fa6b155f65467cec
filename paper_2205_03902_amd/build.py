"""Builds libimsp.so (the HIP library behind include/ms.h) for gfx950 in place."""
from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libimsp.so")
SOURCES = [os.path.join(PKG, "csrc", "ms_lib.hip"), os.path.join(PKG, "csrc", "unet_lib.hip"),
           os.path.join(PKG, "csrc", "datagen_lib.hip"), os.path.join(PKG, "csrc", "smd_lib.hip")]
HEADERS = [os.path.join(ROOT, "include", "ms.h"), os.path.join(ROOT, "include", "unet.h"),
           os.path.join(PKG, "csrc", "ms_kernels.hpp"), os.path.join(PKG, "csrc", "fft_lines.hpp"),
           os.path.join(PKG, "csrc", "line_kernels.hpp"), os.path.join(PKG, "csrc", "unet_kernels.hpp"),
           os.path.join(ROOT, "include", "datagen.h"), os.path.join(PKG, "csrc", "datagen_kernels.hpp"),
           os.path.join(ROOT, "include", "smd.h")]
ARCH = "gfx950"
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def command(out: str = LIB) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            # packed FP32 instructions stay disabled in every kernel
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
            "-Wall", "-Wno-unused-result", "-o", out] + SOURCES + [
            # the dense products of the sparse matrix decomposition are rocBLAS GEMMs
            "-L", os.path.join(ROCM, "lib"), "-lrocblas", "-Wl,-rpath," + os.path.join(ROCM, "lib")]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
