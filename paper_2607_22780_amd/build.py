"""Build ``libgrt.so`` (HIP, gfx950) in-tree with hipcc.

Every source is compiled for gfx950 only, with packed-FP32 instructions
disabled (``-packed-fp32-ops``) and IEEE-rounded FP32 division and square
root (hipcc's default, stated explicitly).
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgrt.so")
# walk statistics (grt_walk_stats): the same sources with -DGRT_STATS
STATS_LIB = os.path.join(HERE, "libgrt_stats.so")
SOURCES = ["api.hip", "scene.hip", "trace.hip", "render.hip", "server.hip", "denoise.hip", "mesh.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fhip-fp32-correctly-rounded-divide-sqrt", "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _objs(jobs: int = 4, verbose: bool = False, stats: bool = False):
    build_dir = os.path.join(HERE, "_build", "stats") if stats else os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    inc = ["-I", CSRC, "-I", os.path.join(ROOT, "include")]
    procs, objs = [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(build_dir, src.replace(".hip", ".o"))
        cmd = [HIPCC] + FLAGS + (["-DGRT_STATS"] if stats else []) + inc + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
        while len([p for p, _ in procs if p.poll() is None]) >= jobs:
            time.sleep(0.2)
    for p, src in procs:
        if p.wait() != 0:
            raise RuntimeError(f"hipcc failed on {src}")
    return objs


def build(verbose: bool = False, stats: bool = False) -> str:
    """Build libgrt.so, or with stats the instrumented libgrt_stats.so."""
    t0 = time.time()
    lib = STATS_LIB if stats else LIB
    objs = _objs(verbose=verbose, stats=stats)
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    if verbose:
        print(f"built {lib} in {time.time() - t0:.1f}s", flush=True)
    return lib


if __name__ == "__main__":
    build(verbose=True, stats="--stats" in sys.argv[1:])
