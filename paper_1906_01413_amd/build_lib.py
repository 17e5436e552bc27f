"""Build libriot.so (the HIP C-ABI library) in-tree for gfx950 with hipcc."""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["l96.hip", "linalg.hip", "eig.hip", "riot_api.hip", "tracer.hip", "net.hip"]
LIB = os.path.join(HERE, "libriot.so")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # keep hipcc from forming packed FP32 instructions on its own
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the RIOT library needs ROCm's hipcc to build")


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libriot.so (always recompiles)."""
    os.makedirs(os.path.join(ROOT, "_build"), exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(ROOT, "_build", src.replace(".hip", ".o"))
        cmd = [hipcc(), *[f for f in FLAGS if f != "-shared"], "-c",
               "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
