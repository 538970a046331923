"""Build libodp.so (HIP, gfx950) in-tree with hipcc.

Every translation unit compiles to an object of its own, in parallel (the
stage kernels are split into one unit per precision and dynamics), then one
hipcc line links the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libodp.so")

SOURCES = ["kernels.hip", "runtime.cpp", "plan.cpp", "tune.cpp", "solve.cpp", "serve.cpp", "noalloc.hip"]
# (precision, dynamics id) slices of the stage kernels
SLICES = [(p, d) for p in (32, 64) for d in range(5)]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # every contraction is written out explicitly in the kernels
    "-ffp-contract=off",
    # no packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]


def _units():
    units = []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        units.append((src, os.path.join(OBJ, os.path.splitext(s)[0] + ".o"), []))
    for p, d in SLICES:
        units.append((os.path.join(CSRC, "stage_inst.hip"), os.path.join(OBJ, f"stage_f{p}_d{d}.o"),
                      [f"-DODP_PREC={p}", f"-DODP_DYN={d}"]))
    return units


def build(verbose: bool = False, jobs: int | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    units = _units()
    if jobs is None:
        jobs = max(1, min(len(units), os.cpu_count() or 1, 16))

    def compile_one(u):
        src, obj, defs = u
        cmd = [hipcc] + FLAGS + defs + ["-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        return cmd, res

    failed = []
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for cmd, res in ex.map(compile_one, units):
            out = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l)
            if out.strip():
                print(out, file=sys.stderr, flush=True)
            if res.returncode != 0:
                failed.append(" ".join(cmd))
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [u[1] for u in units] + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
