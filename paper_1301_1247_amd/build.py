"""Build the HIP library libqpscatter.so for gfx950 in-tree (hipcc, no JIT cache).

Regenerates the Hankel coefficient tables when the generator is newer than the table.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqpscatter.so")

SOURCES = ["kernels_build.hip", "gemm.hip", "kernels_qp.hip", "runtime.cpp", "hbs.cpp", "qp.cpp", "capi.cpp"]

FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-Wno-unused-command-line-argument"]


def _tables():
    gen = os.path.join(CSRC, "gen_hankel_tables.py")
    inc = os.path.join(CSRC, "hankel_tables.inc")
    if not os.path.exists(inc) or os.path.getmtime(gen) > os.path.getmtime(inc):
        out = subprocess.run([sys.executable, gen], check=True, capture_output=True, text=True).stdout
        with open(inc, "w") as f:
            f.write(out)


def build(verbose: bool = False) -> str:
    _tables()
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = []
    for s in SOURCES:
        path = os.path.join(CSRC, s)
        srcs += (["-x", "hip", path] if s.endswith(".cpp") else [path])
    tmp = LIB + ".tmp"
    cmd = [hipcc] + FLAGS + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
