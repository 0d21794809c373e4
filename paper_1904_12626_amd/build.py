"""Build libmpx.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Every translation unit is compiled for gfx950 only, with packed-FP32 VALU
instructions disabled; the sweep unit is built without NaN semantics (its
minima run on packed keys that are never NaN, and that lets the compiler use
plain v_min instructions without canonicalising their inputs).
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmpx.so")
OBJ = os.path.join(HERE, "_build")

SOURCES = {
    "mp_prep.hip": [],
    "mp_sweep.hip": ["-fno-honor-nans"],
    "mp_post.hip": [],
    "mp_backward.hip": [],
    "mp_scan.hip": [],
    "mp_mine.hip": [],
    "mp_md.hip": [],
    "mp_stream.hip": [],
    "mp_abi.cpp": [],
}

COMMON = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-x", "hip",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    hipcc = _hipcc()

    def compile_one(item):
        name, extra = item
        src = os.path.join(CSRC, name)
        obj = os.path.join(OBJ, name + ".o")
        cmd = [hipcc, *COMMON, *extra, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {name}:\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES.items()))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
