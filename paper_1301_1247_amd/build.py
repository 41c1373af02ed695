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

SOURCES = ["kernels_build.hip", "gemm.hip", "gemm_tune.cpp", "kernels_qp.hip", "kernels_mlp.hip", "runtime.cpp",
           "hbs.cpp", "qp.cpp", "wood.cpp", "capi.cpp", "noalloc.cpp"]
MODEL = os.path.join(HERE, "rank_mlp_default.json")
TUNE = os.path.join(HERE, "gemm_tune_default.json")

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


def _model():
    """Embed the trained rank-predictor parameters (rank_mlp_default.json) as a C array."""
    inc = os.path.join(CSRC, "rank_mlp_default.inc")
    if os.path.exists(MODEL):
        import json
        with open(MODEL) as f:
            params = json.load(f)["params"]
        body = ",\n".join(", ".join(f"{float(v):.9e}f" for v in params[i:i + 8]) for i in range(0, len(params), 8))
        text = (f"static const float kRankModelDefault[] = {{\n{body}\n}};\n"
                f"static const int kRankModelDefaultN = {len(params)};\n")
    else:
        text = "static const float kRankModelDefault[1] = {0.0f};\nstatic const int kRankModelDefaultN = 0;\n"
    old = open(inc).read() if os.path.exists(inc) else None
    if old != text:
        with open(inc, "w") as f:
            f.write(text)


def _tune_table():
    """Embed the GEMM tile tuning table (gemm_tune_default.json, written by tune_gemm.py) as a C array."""
    inc = os.path.join(CSRC, "gemm_tune_default.inc")
    pairs = []
    if os.path.exists(TUNE):
        import json
        with open(TUNE) as f:
            pairs = [(int(e["key"]), int(e["cfg"])) for e in json.load(f)["table"]]
    if pairs:
        body = ",\n".join(f"{k}, {c}" for k, c in pairs)
        text = (f"static const int kGemmTuneDefault[] = {{\n{body}\n}};\n"
                f"static const int kGemmTuneDefaultN = {len(pairs)};\n")
    else:
        text = "static const int kGemmTuneDefault[2] = {0, 0};\nstatic const int kGemmTuneDefaultN = 0;\n"
    old = open(inc).read() if os.path.exists(inc) else None
    if old != text:
        with open(inc, "w") as f:
            f.write(text)


def build(verbose: bool = False) -> str:
    _tables()
    _model()
    _tune_table()
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
