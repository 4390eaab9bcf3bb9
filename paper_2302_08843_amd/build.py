"""Build the HIP library libmmx.so (gfx950) in-tree with hipcc.

Usage: python -m paper_2302_08843_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmmx.so")
SOURCES = ["kernels.hip", "mid_f32.hip", "mid_f64.hip", "passes_f32.hip", "passes_f64.hip",
           "local_ext_f32.hip", "local_ext_f64.hip", "api.hip", "serve.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, jobs: int = 0, out: str = LIB, defines=()) -> str:
    """Compile every source to an object and link the library (libmmx.so by
    default); always rebuilds.  `defines` are extra -D flags (tuning knobs)."""
    if jobs <= 0:
        jobs = max(1, min(len(SOURCES), os.cpu_count() or 1, 8))
    tmp = tempfile.mkdtemp(prefix="mmx_build_")
    try:
        objs = []
        procs = []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            cmd = [HIPCC, *FLAGS, *["-D" + d for d in defines], "-c", os.path.join(CSRC, src),
                   "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((subprocess.Popen(cmd), src))
            objs.append(obj)
            if len(procs) >= jobs:
                p, s = procs.pop(0)
                if p.wait() != 0:
                    raise RuntimeError("hipcc failed on " + s)
        for p, s in procs:
            if p.wait() != 0:
                raise RuntimeError("hipcc failed on " + s)
        out_tmp = out + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out_tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out_tmp, out)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
