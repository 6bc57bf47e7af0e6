"""Build libradtex.so (HIP, gfx950) in-tree with hipcc.

Every kernel is compiled for gfx950 only, at -O3, with IEEE-correct binary32
division and square root (HIP's default) and with packed-FP32 instruction
selection disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libradtex.so")
SOURCES = ["rt_abi.cpp", "rt_lookup.hip", "rt_quantize.hip", "rt_backward.hip", "rt_bake.hip",
           "rt_mip.hip", "rt_dictionary.hip", "rt_lod_backward.hip", "rt_noalloc.hip"]
ARCH = os.environ.get("RADTEX_ARCH", "gfx950")


def build(verbose: bool = False, jobs: int = 4, csrc: str = CSRC, lib: str = LIB) -> str:
    """Compile the sources in `csrc` into the shared library `lib`."""
    objdir = os.path.join(os.path.dirname(lib), "_build")
    os.makedirs(objdir, exist_ok=True)
    common = ["hipcc", "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-fno-gpu-rdc", "-Wall", "-Wno-unused-result",
              "-I", os.path.join(ROOT, "include"), "-I", csrc]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src.rsplit(".", 1)[0] + ".o")
        cmd = common + ["-x", "hip", "-c", os.path.join(csrc, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
        if len(procs) >= jobs:
            if procs.pop(0).wait() != 0:
                raise RuntimeError("hipcc failed")
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    link = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", lib + ".tmp"] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    # optional: python build.py <csrc dir> <output library>
    if len(sys.argv) == 3:
        build(verbose=False, csrc=os.path.abspath(sys.argv[1]), lib=os.path.abspath(sys.argv[2]))
    else:
        build(verbose=True)
    sys.exit(0)
