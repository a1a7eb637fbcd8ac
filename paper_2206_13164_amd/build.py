"""Build the gfx950 shared library ``libnrxx.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnrxx.so")
SOURCES = ["nrxx_kernels.hip", "nrxx_batch.hip", "nrxx_api.cpp", "nrxx_batch_api.cpp", "nrxx_mlp.hip",
           "nrxx_noalloc.cpp", "nrxx_wsweep.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are disabled for every HIP translation unit
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # contract a*b+c into FMA only within one source expression, so the same
    # cell arithmetic rounds the same way in every kernel it is inlined into
    # (the sweep schedules are compared bit for bit)
    "-ffp-contract=on",
    "-Wno-unused-command-line-argument",
]


# Per-file extra flags.  The wavefront-per-cell sweep keeps many cells in
# flight per CU only while its register footprint stays small; machine-level
# loop-invariant code motion hoists lane-dependent address arithmetic out of
# its cell loops and roughly doubles that footprint, so it is off there.
EXTRA = {"nrxx_wsweep.hip": ["-mllvm", "-disable-machine-licm"]}


def build(verbose: bool = False) -> str:
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, src + ".o")
        cmd = [HIPCC, *FLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd.insert(1, "-xhip")
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for cmd, p in procs:  # translation units compile in parallel
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, cmd)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
