"""Build libgofmm.so in-tree for gfx950 (hipcc for device code, clang++ with
OpenMP for host code).  `python -m paper_1707_00164_amd.build` or build()."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libgofmm.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")
ARCH = "gfx950"

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
HIP_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             ]
HOST_FLAGS = ["-fopenmp", "-march=x86-64-v2"]


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + p.stdout + p.stderr)
    return p


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    jobs = []
    for f in sorted(os.listdir(SRC)):
        src = os.path.join(SRC, f)
        obj = os.path.join(OUT, f + ".o")
        if f.endswith(".hip"):
            jobs.append([HIPCC] + COMMON + HIP_FLAGS + ["-c", src, "-o", obj])
        elif f.endswith(".cpp"):
            jobs.append([CLANG] + COMMON + HOST_FLAGS + [f"-I{ROCM}/include", "-c", src, "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for p in ex.map(_run, jobs):
            if verbose and (p.stdout or p.stderr):
                print(p.stdout + p.stderr, file=sys.stderr)
    objs = [j[-1] for j in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fopenmp", "-o", tmp] + objs +
         [f"-Wl,-rpath,{ROCM}/llvm/lib", f"-Wl,-rpath,{ROCM}/lib"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
