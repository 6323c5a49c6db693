"""Build libbfly.so (HIP, gfx950) in-tree.

    python -m paper_1305_4650_amd.build

compiles csrc/*.hip and csrc/*.cpp with hipcc into paper_1305_4650_amd/libbfly.so.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbfly.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # tau is taken modulo 1 after reaching ~1e3 turns: its rounding is part of
    # the specification, so no operation may be fused implicitly.
    "-ffp-contract=off",
    # packed FP32 instructions are not used (compiler-formed v_pk_* FP32 ops
    # are avoided on this target)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]
SOURCES = ["bfly_d2.hip", "bfly_d2_batch.hip", "bfly_d3.hip", "bfly_d3_batch.hip", "bfly_d1.hip",
           "bfly_d1_batch.hip", "bfly_common.hip", "bfly_api.cpp", "bfly_timing.cpp", "bfly_phase.hip", "bfly_tune.cpp"]


def build(verbose: bool = True, jobs: int = 6, out: str = LIB, defines=(), build_dir: str = BUILD) -> str:
    """Compile every source (always) and link libbfly.so (or `out`)."""
    os.makedirs(build_dir, exist_ok=True)
    t0 = time.time()
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = [HIPCC, *COMMON, *[f"-D{d}" for d in defines], "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        if len(procs) >= jobs:
            _wait(procs)
    _wait(procs)
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    if verbose:
        print(f"built {out} in {time.time() - t0:.1f}s", flush=True)
    return out


def _wait(procs):
    while procs:
        src, p = procs.pop(0)
        if p.wait() != 0:
            raise RuntimeError(f"hipcc failed on {src}")


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
