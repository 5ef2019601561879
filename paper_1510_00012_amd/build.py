"""Build libd2.so (the HIP library behind include/d2.h) for gfx950, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libd2.so")
SOURCES = ["d2_k_f64.hip", "d2_k_f64w.hip", "d2_k_f32.hip", "d2_k_f32w.hip",
           "d2_k_f64p.hip", "d2_k_f32p.hip", "d2_api.hip", "d2_ws.hip",
           "d2_noalloc.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++20", "-fPIC", "-shared", "--offload-arch=gfx950",
    # keep packed-FP32 instructions out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wno-unused-result",
]


OBJ_DIR = os.path.join(HERE, "_build")


def build(verbose: bool = False) -> str:
    """Compile each translation unit in parallel, then link libd2.so."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs, procs = [], []
    cflags = [f for f in FLAGS if f != "-shared"]
    for src in SOURCES:
        obj = os.path.join(OBJ_DIR, src.replace(".hip", ".o"))
        cmd = [HIPCC, *cflags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for p, cmd in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, cmd)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o",
           tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
