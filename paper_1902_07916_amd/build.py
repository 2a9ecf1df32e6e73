"""Build the gfx950 HIP library ``libzmc.so`` in-tree.

    python -m paper_1902_07916_amd.build [--jobs N]

Compiles the sampling kernel once per integrand (-DZMC_F=<id>), the level
kernels, the engine and the C ABI with hipcc for gfx950, in parallel, and
links them into ``paper_1902_07916_amd/libzmc.so``.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libzmc.so")
N_INTEGRANDS = 8

HIP_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    "-I" + INCLUDE, "-I" + CSRC,
    # no packed FP32 instructions (v_pk_*_f32) anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _units():
    units = []
    for f in range(N_INTEGRANDS):
        units.append((os.path.join(CSRC, "zmc_sample.hip"), os.path.join(BUILD, f"zmc_sample_{f}.o"),
                      [f"-DZMC_F={f}"]))
    # the per-cube / per-integral kernels round every product and sum
    # separately, in the order the method states them (no FMA contraction)
    units.append((os.path.join(CSRC, "zmc_level.hip"), os.path.join(BUILD, "zmc_level.o"), ["-ffp-contract=off"]))
    for name in ("zmc_engine", "zmc_abi"):
        units.append((os.path.join(CSRC, name + ".hip"), os.path.join(BUILD, name + ".o"), []))
    return units


def _compile(src, obj, extra):
    cmd = [hipcc()] + HIP_FLAGS + extra + ["-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(cmd), res.stdout, res.stderr))
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every translation unit and link libzmc.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    units = _units()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, *u) for u in units]
        objs = [f.result() for f in futs]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed: %s\n%s%s" % (" ".join(cmd), res.stdout, res.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    a = ap.parse_args(argv)
    build(a.jobs, verbose=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
