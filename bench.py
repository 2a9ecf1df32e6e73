"""Benchmark: integrand samples/s of the whole tree search on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sin6d|gauss9d|gauss4d]

One step is one complete integration (every level: sampling, per-cube
reduction, threshold, selection, subdivision) of the workload, with all
inputs resident on the device.  Default workload: the paper's f1 =
sin(sum_{i=1..6} x_i) on [0,10]^6 with 6 divisions per axis (46656 root
cubes), 16384 points per cube, 5 trials, two refinement levels, sigma 1,
evaluated in FP32 with FP64 sums.  The plain FP64 path is timed beside it,
and the CPU oracle on a bounded sample of the same workload.

Prints one JSON line (see the repository's design notes for every field).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X figures used by the roofline (vendor specification)
N_CU = 256
CLOCK_HZ = 2.4e9
LANES_PER_CU_CLK = 64            # 4 SIMDs x 16 lanes: one wave64 VALU op per SIMD per 4 clocks
VALU_PEAK = N_CU * CLOCK_HZ * LANES_PER_CU_CLK   # 3.93e13 lane-cycles/s
FP32_PEAK_FLOPS = 157.3e12       # packed FP32 FMA
FP64_PEAK_FLOPS = 78.6e12

# Issue cost, in lane-cycles per lane, of the instruction forms the sampling
# kernel needs (quarter-rate ops take 4); measured on gfx950 with a
# throughput probe (see the design notes).
COST = dict(mad_u64=4.0, bitop3=1.0, alu=1.0, fma32=1.0, trans32=4.0, fp64=1.0)


def valu_cycles_per_sample(integrand: str, D: int, eval_: str) -> dict:
    """Minimal VALU lane-cycles per sample of the method on this ISA.

    RNG: D/4 Philox4x32-10 blocks per sample; a block is 10 rounds of two
    32x32->64 products and two 3-input XORs, of which the first round's
    product of the (wave-uniform) counter word 2 and its XOR are scalar work
    -> 18 v_mad_u64_u32 + 18 v_bitop3_b32 per block.  Map: one bit-op per
    coordinate (+ the FMA that places it in the cube).  Integrand and the
    FP64 accumulation (f, f^2) as listed per family."""
    blocks = D / 4.0
    rng = blocks * (18 * COST["mad_u64"] + 18 * COST["bitop3"])
    if eval_ == "fp32":
        mapping = D * (COST["alu"] + COST["fma32"])
        if integrand == "sin_sum":
            f = 13 * COST["alu"]                       # sin(2 pi r) reduction + odd polynomial
        elif integrand == "gauss":
            f = D * COST["fma32"] + COST["fma32"] + COST["trans32"] + COST["fma32"]  # t^2 sum, scale, exp2, A*
        else:
            f = 2 * D * COST["fma32"] + COST["trans32"]
        acc = 3 * COST["fp64"]                         # cvt, add, fma
        flops32 = 2 * D + (16 if integrand == "sin_sum" else 2 * D + 2)
    else:
        mapping = D * (3 * COST["alu"] + COST["fp64"])  # shift/or, cvt, fma
        f = (D + 30) * COST["fp64"]                    # sum + FP64 sin / exp
        acc = 2 * COST["fp64"]
        flops32 = 0
    return dict(rng=rng, map=mapping, f=f, acc=acc, total=rng + mapping + f + acc, fp32_flops=flops32)


WORKLOADS = {
    "sin6d": ("sin6d", "sin_sum", "f1 = sin(sum x_i) on [0,10]^6, d=6 (46656 root cubes), N=16384, n1=5, "
              "max_depth=2, sigma_mult=1, seed=1"),
    "gauss9d": ("narrow_gauss9d", "gauss", "prod exp(-(x_i-0.5)^2/(2*0.02^2)) on [0,1]^9, d=3 (19683 cubes), "
                "N=65536, n1=5, max_depth=3, sigma_mult=0.5, seed=1"),
    "gauss4d": ("gauss4d", "gauss", "exp(-|x|^2/(2*0.2^2)) on [-1,1]^4, d=4 (256 cubes), N=4096, n1=5, "
                "max_depth=1, sigma_mult=1, seed=1"),
}


def cpu_baseline(w: dict, seconds: float) -> dict:
    """The CPU oracle as it stands, single thread, on the first root cubes of
    the same workload (all trials, all points), until `seconds` elapse."""
    import oracle
    p = oracle.problem(w["integrand"], len(w["lower"]), w["lower"], w["upper"], w["divisions"], w["samples"],
                       w["trials"], w["max_depth"], w["sigma_mult"], w["seed"], params=w["params"])
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds:
        oracle.cube(p, 0, n)
        n += 1
    dt = time.perf_counter() - t0
    samples = n * w["trials"] * w["samples"]
    return {"value": samples / dt, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": "level-0 cubes 0..%d of the same workload, %d trials x %d points each (%.3g samples, %.1f s)"
                      % (n - 1, w["trials"], w["samples"], samples, dt)}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sin6d", choices=sorted(WORKLOADS))
    ap.add_argument("--no-fp64", action="store_true", help="skip timing the plain FP64 path")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--arena-gib", type=float, default=48.0)
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the work would shard by whole "
              "integrals or by contiguous uid ranges with one small all-reduce per level); run with --gpus 1",
              file=sys.stderr)
        return 2

    import torch
    from paper_1902_07916_amd import Integrator, workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    gen, integrand, desc = WORKLOADS[a.workload]
    w32 = getattr(workloads, gen)(eval="fp32")
    w64 = getattr(workloads, gen)(eval="fp64")
    D = len(w32["lower"])
    zi = Integrator(arena_bytes=int(a.arena_gib * (1 << 30)))

    for _ in range(a.warmup):
        zi.integrate(**w32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [zi.integrate(**w32) for _ in range(a.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    samples = sum(r.n_samples for r in results)
    value = samples / dt
    r = results[-1]

    # dominant kernel: the sampling kernel, timed with HIP events on its stream
    k_ms = sum(sum(x.sample_ms_per_level) for x in results)
    k_launches = sum(sum(x.sample_launches_per_level) for x in results)
    k_samples = samples
    cyc = valu_cycles_per_sample(integrand, D, "fp32")
    achieved = k_samples * cyc["total"] / (k_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK, "unit": "VALU lane-cycles/s",
                "frac": achieved / VALU_PEAK, "traffic": None,
                "kernel": "sample_kernel<%s,D=%d,FP32>" % (integrand, D),
                "avg_launch_ms": k_ms / max(k_launches, 1), "launches": k_launches,
                "cycles_per_sample": cyc, "kernel_samples_per_s": k_samples / (k_ms * 1e-3),
                "fp32_flop_frac": k_samples * cyc["fp32_flops"] / (k_ms * 1e-3) / FP32_PEAK_FLOPS}

    out = {"metric": "integrand samples/sec + % FP32 VALU peak vs plain FP64; p50/p99 latency at QPS",
           "value": value, "unit": "samples/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": dt * 1e3 / a.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": a.workload + ": " + desc + "; integrand in FP32, sums/threshold in FP64",
                      "levels": r.cubes_per_level, "selected": r.selected_per_level,
                      "samples_per_step": r.n_samples},
           "result": {"integral": r.integral, "stderr": r.stderr, "std": r.std},
           "roofline": roofline}
    if a.workload == "sin6d":
        exact = -49.16507381641946
        out["result"]["exact"] = exact
        out["result"]["z"] = (r.integral - exact) / r.stderr

    if not a.no_fp64:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r64 = zi.integrate(**w64)
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t0
        out["fp64_path"] = {"value": r64.n_samples / dt64, "unit": "samples/s", "ms_per_step": dt64 * 1e3,
                            "integral": r64.integral, "stderr": r64.stderr, "levels": r64.cubes_per_level,
                            "speedup_fp32_over_fp64": value / (r64.n_samples / dt64),
                            "rel_diff_fp32_vs_fp64": abs(r.integral - r64.integral) / abs(r64.integral)}
    zi.close()
    if a.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(w64, a.cpu_seconds)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
