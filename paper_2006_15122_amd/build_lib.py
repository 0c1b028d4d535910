"""Build the HIP library libcosmolat.so for gfx950 (hipcc, in-tree).

Each source is compiled to an object in parallel, then the objects are
linked into the shared library next to this file."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["lattice.hip", "scalar.hip", "fft.hip", "u1.hip", "su2.hip", "noalloc.hip", "batch.hip", "mlp.hip"]
OUT = os.path.join(HERE, "libcosmolat.so")
HIPCC = "/opt/rocm/bin/hipcc"

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-value",
]


def build(verbose: bool = False) -> str:
    with tempfile.TemporaryDirectory(prefix="cosmolat_build_") as td:
        procs, objs = [], []
        for s in SOURCES:
            obj = os.path.join(td, s + ".o")
            cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, s), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((cmd, subprocess.Popen(cmd)))
            objs.append(obj)
        failed = [cmd for cmd, p in procs if p.wait() != 0]
        if failed:
            raise subprocess.CalledProcessError(1, failed[0])
        tmp = OUT + ".tmp"
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
        os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
