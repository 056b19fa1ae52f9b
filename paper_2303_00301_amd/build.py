"""Build libauxkf.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libauxkf.so")
ARCH = os.environ.get("AKF_OFFLOAD_ARCH", "gfx950")
SOURCES = ["akf_kernels.hip", "akf_adjoint.hip", "akf_fact.hip", "akf_dyn.hip", "akf_dnc.hip",
           "akf_fixed.hip", "akf_gibbs.hip", "akf_noalloc.hip", "akf_sqrt.hip", "akf_lane.hip",
           "akf_layout.cpp", "akf_capi.cpp", "akf_batch.cpp"]
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (in parallel, `jobs` at a time; 0 = one per CPU up
    to 16) and link libauxkf.so in place."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    jobs = jobs or max(1, min(16, os.cpu_count() or 1))
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, src + ".o")
        cmds.append([hipcc, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for rc, cmd in zip(ex.map(lambda c: subprocess.call(c), cmds), cmds):
            if rc != 0:
                raise subprocess.CalledProcessError(rc, cmd)
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
