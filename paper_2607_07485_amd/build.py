"""Build liblsdd.so (HIP kernels for gfx950 + host driver) in-tree.

    python -m paper_2607_07485_amd.build [--jobs N]

Produces paper_2607_07485_amd/liblsdd.so; objects go to paper_2607_07485_amd/_build/.
"""
from __future__ import annotations

import argparse
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "liblsdd.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = os.environ.get("LSDD_ARCH", "gfx950")

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep hand-written and compiler-formed packed FP32 ops out of the code objects
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
]
CXX_FLAGS = [
    "-O2", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", f"-I{os.path.join(ROCM, 'include')}",
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(jobs: int = 4, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    steps = [
        [hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, "kernels.hip"), "-o", os.path.join(BUILD, "kernels.o")],
        [hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, "batched.hip"), "-o", os.path.join(BUILD, "batched.o")],
        [hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, "blk.hip"), "-o", os.path.join(BUILD, "blk.o")],
        [hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, "trd.hip"), "-o", os.path.join(BUILD, "trd.o")],
        [hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, "noalloc.hip"), "-o", os.path.join(BUILD, "noalloc.o")],
        ["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, "lsdd.cpp"), "-o", os.path.join(BUILD, "lsdd.o")],
        ["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, "graph.cpp"), "-o", os.path.join(BUILD, "graph.o")],
    ]
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for r in ex.map(_run, steps):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr)
    objs = [os.path.join(BUILD, f) for f in ("kernels.o", "batched.o", "blk.o", "trd.o", "noalloc.o", "lsdd.o",
                                             "graph.o")]
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp,
          f"-L{os.path.join(ROCM, 'lib')}", "-lamdhip64", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}",
          "-Wl,--no-undefined"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.verbose))
