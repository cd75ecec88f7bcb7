"""Build libspeedysplat.so for gfx950 with hipcc (in-tree, no JIT cache).

    python -m paper_2412_00578_amd.csrc.build            # build
    python -m paper_2412_00578_amd.csrc.build --asm      # also dump gfx950 ISA

Flags: -O3, -ffp-contract=off (every FP64/FP32 op rounded once in the written
order; the geometry is reproducible bit for bit), packed-FP32 instructions
disabled, position-independent code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libspeedysplat.so")
SOURCES = ["api.hip", "k_preprocess.hip", "k_scan.hip", "k_emit.hip", "k_sort.hip",
           "k_tile_order.hip", "k_blend.hip", "k_backward.hip", "k_prune.hip"]
ARCH = os.environ.get("SS_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def common_flags():
    return ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-ffp-contract=off",
            "-munsafe-fp-atomics",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


def _compile(src: str, obj_dir: str) -> str:
    obj = os.path.join(obj_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *common_flags(), "-c", os.path.join(HERE, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    obj_dir = os.path.join(ROOT, "_build", "obj")
    os.makedirs(obj_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, obj_dir), SOURCES))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def dump_asm(out_dir: str) -> None:
    os.makedirs(out_dir, exist_ok=True)
    for src in SOURCES:
        out = os.path.join(out_dir, os.path.splitext(src)[0] + ".s")
        cmd = [hipcc(), *common_flags(), "--cuda-device-only", "-S",
               os.path.join(HERE, src), "-o", out]
        subprocess.run(cmd, check=True)


if __name__ == "__main__":
    build(verbose=True)
    if "--asm" in sys.argv:
        dump_asm(os.path.join(ROOT, "_build", "asm"))
