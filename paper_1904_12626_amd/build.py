"""Build libmpx.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Every translation unit is compiled for gfx950 only, with packed-FP32 VALU
instructions disabled; the sweep unit is built without NaN semantics (its
minima run on packed keys that are never NaN, and that lets the compiler use
plain v_min instructions without canonicalising their inputs).
"""

from __future__ import annotations

import hashlib
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmpx.so")
OBJ = os.path.join(HERE, "_build")
# SHA-256 of the FP32 sweep kernels' gfx950 assembly as built (the function
# bodies of every k_sweep<float, ...> instantiation, compilation-unit ids left
# out), which ties recorded hardware counters to the code they were taken on
SWEEP_ISA = os.path.join(HERE, "libmpx.sweep.sha256")

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


# Issue-rate probe of the sweep's VALU instruction mix (bench.py runs it and
# reports the sweep against the rate it measures)
PROBE_SRC = os.path.join(ROOT, "bench_valu.hip")
PROBE = os.path.join(OBJ, "bench_valu")


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

    def sweep_isa():
        out = os.path.join(OBJ, "mp_sweep.gfx950.s")
        cmd = [hipcc, *COMMON, *SOURCES["mp_sweep.hip"], "--cuda-device-only", "-S",
               os.path.join(CSRC, "mp_sweep.hip"), "-o", out]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc -S failed for mp_sweep.hip:\n{r.stdout}\n{r.stderr}")
        h = hashlib.sha256()
        inside = False
        with open(out, "rb") as f:
            for line in f.read().split(b"\n"):
                if re.match(rb"^_ZN3mpx7k_sweepIf\w*:", line):
                    inside = True
                if inside:
                    if not (b"__hip_cuid" in line or line.lstrip().startswith((b".file", b".ident"))):
                        h.update(line + b"\n")
                    if line.startswith(b".Lfunc_end"):
                        inside = False
        return h.hexdigest()

    def probe():
        cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
               "-packed-fp32-ops", "-Wno-unused-command-line-argument", PROBE_SRC, "-o", PROBE]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for bench_valu.hip:\n{r.stdout}\n{r.stderr}")

    with ThreadPoolExecutor(max_workers=len(SOURCES) + 2) as ex:
        isa = ex.submit(sweep_isa)
        prb = ex.submit(probe)
        objs = list(ex.map(compile_one, SOURCES.items()))
        isa_hash = isa.result()
        prb.result()
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    with open(SWEEP_ISA, "w") as f:
        f.write(isa_hash + "\n")
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
