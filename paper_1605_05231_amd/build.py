"""Build libnufftct.so (HIP kernels for gfx950 + the C-ABI) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libnufftct.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["plan.cpp", "host_plan.cpp", "tables.cpp", "batch.cpp", "umbrella.cpp", "grangeat.cpp",
           "k_fft_f32.hip", "k_fft_f64.hip", "k_grid_f32.hip", "k_grid_f64.hip", "k_umbrella.hip",
           "k_resample1_f32.hip", "k_resample1_f64.hip", "k_grangeat_f32.hip", "k_grangeat_f64.hip",
           "k_batch_f32.hip", "k_batch_f64.hip"]

ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          # packed FP32 instructions are disabled for every HIP translation unit
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-Wno-unused-command-line-argument"]
HOST_ONLY = {"plan.cpp": ["-ffp-contract=off"], "host_plan.cpp": ["-ffp-contract=off"],
             "tables.cpp": ["-ffp-contract=off"],
             "batch.cpp": [], "umbrella.cpp": [], "grangeat.cpp": []}


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str, verbose: bool, build_dir: str) -> str:
    obj = os.path.join(build_dir, src + ".o")
    cmd = [hipcc(), "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + HOST_ONLY.get(src, [])
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int | None = None, out: str | None = None) -> str:
    out = out or OUT
    build_dir = BUILD if out == OUT else out + ".objs"
    os.makedirs(build_dir, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, build_dir), SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if a != "-v"]
    print(build(verbose="-v" in sys.argv, out=args[0] if args else None))
