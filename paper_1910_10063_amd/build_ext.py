"""Compile the HIP sources of this package for gfx950 into in-tree shared libraries.

    python -m paper_1910_10063_amd.build_ext

libskew.so     the C ABI of include/skew.h (layout build and query kernels)
libskewgen.so  the seeded workload generator (device half)
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
OBJDIR = os.path.join(HERE, "lib", "obj")
ROOT = os.path.dirname(HERE)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # no packed fp32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{os.path.join(ROOT, 'include')}",
]

TARGETS = {
    "libskew.so": ["skew_api.hip", "layout_kernels.hip", "partition_kernels.hip", "join_kernels.hip",
                   "group_kernels.hip", "operator_kernels.hip", "model_kernels.hip", "star_kernels.hip",
                   "probe_kernels.hip"],
    "libskewgen.so": ["workload_gen.hip"],
}


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> dict:
    """Compile every HIP source (always) and link the libraries into lib/."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sorted({s for v in TARGETS.values() for s in v})
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = dict(zip(srcs, ex.map(_compile, srcs)))
    out = {}
    for lib, parts in TARGETS.items():
        path = os.path.join(LIBDIR, lib)
        tmp = path + f".tmp{os.getpid()}"
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *[objs[p] for p in parts]]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed for {lib}:\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, path)
        out[lib] = path
        if verbose:
            print("built", path)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
