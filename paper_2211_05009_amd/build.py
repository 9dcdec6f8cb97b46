"""Build the gfx950 HIP library in-tree: ``paper_2211_05009_amd/liblbm.so``.

    python paper_2211_05009_amd/build.py

(run as a file: importing the package would load the library being built).

hipcc cross-compiles for gfx950 without a GPU.  Packed-FP32 instruction
selection is disabled (-packed-fp32-ops) for every device compilation, and
multiply-adds are fused only within one source expression (-ffp-contract=on),
so every kernel variant that evaluates the same expressions rounds the same
way.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbm.so")
ARCH = "gfx950"

SOURCES = ["lbm.hip", "lbm_batch.hip", "lbm_nn.hip", "lbm_series.hip", "lbm3d.hip"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]
OBJ_DIR = os.path.join(PKG, "_build")


def compile_command(src: str, obj: str) -> list:
    return [hipcc()] + FLAGS + ["-c", "-o", obj, os.path.join(CSRC, src)]


def link_command(objs: list, out: str = LIB) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-shared", "-o", out] + objs


def _run(cmd: list, verbose: bool) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with exit code {res.returncode}: {' '.join(cmd)}")


def build_library(verbose: bool = False) -> str:
    """Compile every HIP source (in parallel, one object each) and link
    liblbm.so (always recompiles)."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs = [os.path.join(OBJ_DIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    jobs = min(len(SOURCES), max(1, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        for f in [pool.submit(_run, compile_command(s, o), verbose)
                  for s, o in zip(SOURCES, objs)]:
            f.result()
    tmp = LIB + ".tmp"
    _run(link_command(objs, tmp), verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
