"""Build ``libfluxlbm.so`` in-tree with hipcc for gfx950.

Run as ``python -m paper_1806_10589_amd.build`` or through
``__graft_entry__.build()``. Always recompiles.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfluxlbm.so")
SOURCES = [os.path.join(HERE, "csrc", s) for s in ("engine.hip", "mlp.hip", "lattice.cpp")]
ARCH = os.environ.get("FLBM_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    # gfx950: keep the compiler from forming packed FP32 (v_pk_*_f32) ops.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # Keep instructions common to the branches of a step kernel's tile forms
    # (8-bit, 16-bit codes, int32 rows) in each branch: sunk into the join,
    # the last direction's gather waited there for every gather before it,
    # one memory round trip per wave (FP16 step 131.5 -> 129.4 us).
    "-mllvm", "-simplifycfg-sink-common=false",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    path = os.path.join(rocm, "bin", "hipcc")
    return path if os.path.exists(path) else "hipcc"


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libfluxlbm.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
