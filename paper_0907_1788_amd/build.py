"""Builds libfntrs.so in-tree with hipcc for gfx950.

The library is two host translation units (fntrs.hip: C ABI and locator
kernels; submit.hip: batches, graphs, autotuner) plus one translation unit
per transform size for the
compile-time kernels (ct_inst.hip with -DFNTRS_L=1..15), plus the
four-step kernels for n = 2^14 .. 2^16 (fourstep.hip), the 16-bit
transport kernels (wire.hip) and the direct quadratic methods (direct.hip) and the chirp evaluation
(chirp.hip, with one fused kernel per product length in chirp_inst.hip
-DFNTRS_L=1..13).  They compile in
parallel into paper_0907_1788_amd/_build/ and link into libfntrs.so.

Usage: python -m paper_0907_1788_amd.build   (or call build()).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "libfntrs.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SIZES = range(1, 16)
CHIRP_SIZES = range(1, 14)   # fused chirp products of 2^1 .. 2^13 points

FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    "--offload-arch=gfx950",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return res.stderr


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every HIP translation unit and link the shared library."""
    os.makedirs(BUILD, exist_ok=True)
    units = [(os.path.join(CSRC, "fntrs.hip"), os.path.join(BUILD, "fntrs.o"), []),
             (os.path.join(CSRC, "submit.hip"), os.path.join(BUILD, "submit.o"), []),
             (os.path.join(CSRC, "fourstep.hip"), os.path.join(BUILD, "fourstep.o"), []),
             (os.path.join(CSRC, "wire.hip"), os.path.join(BUILD, "wire.o"), []),
             (os.path.join(CSRC, "direct.hip"), os.path.join(BUILD, "direct.o"), []),
             (os.path.join(CSRC, "chirp.hip"), os.path.join(BUILD, "chirp.o"), [])]
    for L in SIZES:
        units.append((os.path.join(CSRC, "ct_inst.hip"), os.path.join(BUILD, f"ct_{L}.o"), [f"-DFNTRS_L={L}"]))
    for L in CHIRP_SIZES:
        units.append((os.path.join(CSRC, "chirp_inst.hip"), os.path.join(BUILD, f"chirp_{L}.o"), [f"-DFNTRS_L={L}"]))
    jobs = jobs or min(16, os.cpu_count() or 4)
    # the large sizes take longest: start them first
    order = sorted(units, key=lambda u: -int(u[2][0].split("=")[1]) if u[2] else 0)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_run, [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]) for src, obj, extra in order]
        logs = [f.result() for f in futs]
    tmp = OUT + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *[u[1] for u in units], "-o", tmp])
    if verbose:
        for l in logs:
            if l.strip():
                print(l)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
