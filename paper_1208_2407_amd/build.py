"""Build libtsq.so (HIP kernels for gfx950 + C-ABI host code) in-tree with hipcc.

Usage: python -m paper_1208_2407_amd.build
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libtsq.so")
ARCH = "gfx950"

COMMON = [
    "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wextra",
    "-ffp-contract=off",            # every fused multiply-add is written out (bitwise-stable order)
    f"-I{os.path.join(ROOT, 'include')}",
]
DEVICE = [
    f"--offload-arch={ARCH}",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libtsq)")


def build(verbose: bool = False, jobs: int = 0, incremental: bool = False) -> str:
    """Compile every csrc/*.hip (device) and csrc/*.cpp (host) file in parallel and
    link libtsq.so.  incremental: skip a source whose object is newer than it and
    than every header (csrc/*.h, *.hpp, include/*.h)."""
    os.makedirs(OUT_DIR, exist_ok=True)
    cc = hipcc()
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip"))) + sorted(glob.glob(os.path.join(CSRC, "*.cpp")))
    headers = (glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(CSRC, "*.hpp"))
               + glob.glob(os.path.join(ROOT, "include", "*.h")))
    newest_header = max((os.path.getmtime(h) for h in headers), default=0.0)
    cmds = []
    objs = []
    for src in srcs:
        obj = os.path.join(OUT_DIR, os.path.basename(src) + ".o")
        objs.append(obj)
        if (incremental and os.path.exists(obj)
                and os.path.getmtime(obj) > max(os.path.getmtime(src), newest_header)):
            continue
        dev = src.endswith(".hip")
        cmds.append([cc, "-c", src, "-o", obj] + COMMON + (DEVICE if dev else []))
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    jobs = jobs or max(1, min(len(cmds), os.cpu_count() or 1, 8))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        for r in ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds):
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError(f"hipcc failed: {' '.join(r.args)}")
    tmp = LIB + ".tmp"
    cmd = [cc, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
