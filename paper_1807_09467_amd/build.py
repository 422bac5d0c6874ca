"""Build the rsolve HIP library (librsolve.so) for gfx950 with hipcc.

Usage: python -m paper_1807_09467_amd.build   (or call build())
Every call recompiles all sources (parallel hipcc processes) into the package
directory, where the binding loads it from.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "librsolve.so")
GEN_OUT = os.path.join(PKG, "libqkgen.so")
BUILD_DIR = os.path.join(PKG, "_build")
SOURCES = ["k_sparse.hip", "k_krylov.hip", "k_dense.hip", "k_eig.hip", "k_ssor.hip", "k_small.hip", "engine.hip",
           "server.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm toolchain required to build librsolve.so)")


def flags():
    return [
        f"--offload-arch={ARCH}",
        "-O3",
        "-std=c++17",
        "-fPIC",
        "-Wall",
        "-Wno-unused-function",
        # packed FP32 instructions are kept out of every kernel
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        f"-I{os.path.join(ROOT, 'include')}",
    ]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()

    def compile_one(src):
        obj = os.path.join(BUILD_DIR, src.replace(".hip", ".o"))
        cmd = [cc, *flags(), "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    _link(cc, objs, OUT)
    # the input generator's own library (finite-element assembly on the GPU)
    gen_src = os.path.join(PKG, "gen_csrc", "qkgen.hip")
    gen_obj = os.path.join(BUILD_DIR, "qkgen.o")
    r = subprocess.run([cc, *flags(), "-c", gen_src, "-o", gen_obj], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for qkgen.hip:\n{r.stdout}\n{r.stderr}")
    _link(cc, [gen_obj], GEN_OUT)
    return OUT


def _link(cc, objs, out):
    tmp = out + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)


if __name__ == "__main__":
    print(build(verbose=True))
