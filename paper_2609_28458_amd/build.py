"""Build the HIP library ``libgradsolve.so`` in-tree for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgradsolve.so")
# The C ABI, and one translation unit of kernels per right-hand side.
SOURCES = [os.path.join(CSRC, f) for f in (
    "gradsolve.hip", "gs_inst_harmonic.hip", "gs_inst_kepler.hip", "gs_inst_loghalo.hip",
    "gs_inst_spinprec.hip", "gs_inst_quint.hip", "gs_inst_stiff.hip")]
HEADERS = [os.path.join(CSRC, h) for h in (
    "gs_kernels.hpp", "gs_rhs.hpp", "gs_tableaux.hpp", "gs_ops.hpp", "gs_inst.hpp",
    "gs_dual.hpp", "gs_de.hpp", "gs_stiff.hpp", "gs_order.hpp")] + [
    os.path.join(ROOT, "include", "gradsolve.h")]
OBJDIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # Every floating-point operation is the one written: fused multiply-adds
    # only where fma() is called, so a replay reproduces the forward pass
    # bit for bit.
    "-ffp-contract=off",
    # No packed FP32 instructions anywhere.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _jobs() -> int:
    for var in ("MAX_JOBS", "CMAKE_BUILD_PARALLEL_LEVEL"):
        v = os.environ.get(var, "")
        if v.isdigit() and int(v) > 0:
            return int(v)
    return max(1, min(len(SOURCES), os.cpu_count() or 1))


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB):
        mt = os.path.getmtime(LIB)
        if all(os.path.getmtime(f) <= mt for f in SOURCES + HEADERS):
            return LIB
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = [os.path.join(OBJDIR, os.path.basename(s)[:-4] + ".o") for s in SOURCES]
    cmds = [[HIPCC, *FLAGS, *inc, "-c", "-o", o, s] for s, o in zip(SOURCES, objs)]
    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        procs = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
    for c, p in zip(cmds, procs):
        if verbose or p.returncode:
            print(" ".join(c), flush=True)
            sys.stdout.write(p.stdout)
            sys.stderr.write(p.stderr)
        if p.returncode:
            raise subprocess.CalledProcessError(p.returncode, c)
    tmp = LIB + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
    sys.exit(0)
