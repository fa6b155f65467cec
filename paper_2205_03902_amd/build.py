"""Builds libimsp.so (the HIP library behind include/ms.h) for gfx950 in place."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

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


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


FLAGS = ["-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions stay disabled in every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"), "-Wall", "-Wno-unused-result"]
LINK = []
OBJ_DIR = os.path.join(ROOT, "_build")


def compile_command(src: str, obj: str) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-c"] + FLAGS + ["-o", obj, src]


def link_command(objs, out: str = LIB) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out] + list(objs) + LINK


def build(verbose: bool = False) -> str:
    """Compiles every source to an object in parallel (one hipcc per source), then links."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs = [os.path.join(OBJ_DIR, os.path.splitext(os.path.basename(s))[0] + ".o") for s in SOURCES]
    cmds = [compile_command(s, o) for s, o in zip(SOURCES, objs)]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    with ThreadPoolExecutor(max_workers=min(len(cmds), max(1, os.cpu_count() or 1))) as ex:
        results = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
    for c, r in zip(cmds, results):
        if r.stderr:
            print(r.stderr, end="", file=sys.stderr, flush=True)
        if r.returncode != 0:
            raise subprocess.CalledProcessError(r.returncode, c)
    tmp = LIB + ".tmp"
    cmd = link_command(objs, tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
