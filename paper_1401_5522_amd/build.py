"""Build libluqr.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

Each translation unit is compiled in parallel into _build/, then linked into
paper_1401_5522_amd/libluqr.so.  Packed FP32 instructions are disabled for
all device code (-Xclang -target-feature -Xclang -packed-fp32-ops).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libluqr.so")
# (source, object name, extra flags): inst.hip once per (precision, tile size)
TILES = {0: (32, 64, 128, 256), 1: (32, 64, 128, 256, 512), 2: (32, 64, 128, 256, 512)}
UNITS = [("api.hip", "api", []), ("batched.hip", "batched", [])] + [
    ("inst.hip", f"inst_p{p}_nb{nb}", [f"-DLQ_P={p}", f"-DLQ_NB={nb}"]) for p, nbs in TILES.items() for nb in nbs]
ARCH = os.environ.get("LUQR_ARCH", "gfx950")

FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")]


def _compile(unit) -> str:
    src, name, extra = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = ["hipcc", *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        msg = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
        raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    units = [u for u in UNITS if os.path.exists(os.path.join(CSRC, u[0]))]
    jobs = min(len(units), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    # the largest tile sizes take longest: start them first
    units.sort(key=lambda u: -int(u[2][1].split("=")[1]) if u[2] else 0)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, units))
    tmp = LIB + ".tmp"
    subprocess.check_call(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
