"""Build libbandops.so (gfx950) from csrc/ with hipcc.

One translation unit per compiled bandwidth (bandops_kern.hip with -DBO_K=k)
plus the host library; compiled in parallel, linked into the package directory.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbandops.so")
KMAX = 12
ARCH = os.environ.get("BANDOPS_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall",
    "-Wno-unused-function", "-Wno-unused-variable",
    # packed FP32 instructions stay off in every HIP object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(HERE, "..", "include"),
]


def _compile(args):
    src, obj, extra = args
    cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    units = []
    for k in range(KMAX + 1):
        units.append((os.path.join(CSRC, "bandops_kern.hip"),
                      os.path.join(BUILD, f"kern_k{k}.o"), [f"-DBO_K={k}"]))
    units.append((os.path.join(CSRC, "bandops_lib.hip"), os.path.join(BUILD, "lib.o"), []))
    units.append((os.path.join(CSRC, "bandops_wide.hip"), os.path.join(BUILD, "wide.o"), []))
    units.append((os.path.join(CSRC, "bandops_graph.hip"), os.path.join(BUILD, "graph.o"), []))
    jobs = jobs or min(len(units), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, units))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(int(sys.argv[1]) if len(sys.argv) > 1 else None)
