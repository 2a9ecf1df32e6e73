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

# MI355X figures used by the roofline (vendor specification: 256 CUs at
# 2.4 GHz; FP32 157.3 TFLOP/s = 128 FMA lanes per CU per clock, i.e. two
# wave64 VALU instructions per SIMD every 4 clocks).
N_CU = 256
CLOCK_HZ = 2.4e9
ISSUE_LANES_PER_CU_CLK = 128
VALU_PEAK = N_CU * CLOCK_HZ * ISSUE_LANES_PER_CU_CLK   # 7.86e13 VALU lane-instructions/s
INT_LANES_PER_CU_CLK = 64   # one integer wave64 instruction per SIMD every 4 clocks (measured 52-66)
FP32_PEAK_FLOPS = 157.3e12
FP64_PEAK_FLOPS = 78.6e12


def valu_instructions_per_sample(integrand: str, D: int, eval_: str) -> dict:
    """Minimal VALU instructions per sample the method needs on this ISA, by
    class (each instruction counts once, whatever its width or pipe).

    RNG: D/4 Philox4x32-10 blocks per sample.  A block is 10 rounds of two
    32x32->64 products and two 3-input XORs; with counter words 1-3 uniform
    over a wave the first round's product of word 2, its XOR and the second
    round's product of word 0 are scalar work: 18 v_mad_u64_u32 + 19
    v_bitop3_b32 per block.  Mapping: one v_alignbit_b32 per coordinate plus
    the FMA that places it.  Integrand per family.  Accumulation: in FP32
    evaluation a lane's 4 values of a group are added in FP32 (3 adds) and
    the group's sum converted and added in FP64 (2 instructions), 0.75 FP32
    and 0.5 FP64 instructions per sample; in FP64, one add.  The sum of squares is kept only on traced
    levels and is not counted."""
    rng = D / 4.0 * 37
    if eval_ == "fp32":
        ints, fp32, fp64, trans = rng + D, float(D) + 0.75, 0.5, 0.0
        if integrand in ("sin_sum", "genz_osc"):
            # high part of the cube phase; r - rint(r) (rint, sub), fold
            # a = min(|t|, 1/2 - |t|) (sub, min), a^2, 6 FMA, *a; the sign
            # back on (copysign, an integer bit-field insert)
            fp32 += 11
            ints += 1
        elif integrand == "gauss":
            fp32 += D + 1          # t^2 sum (from the cube's minimum), scale
            trans += 1             # exp2 (the amplitude multiplies the unit's FP64 sum)
        elif integrand == "genz_gauss":
            fp32 += D              # t^2 sum (from the cube's minimum)
            trans += 1             # exp2 of the negated sum (a source modifier)
        elif integrand == "genz_ppeak":
            fp32 += 2 * D
            trans += 1             # rcp
        else:
            fp32 += 5
            trans += 1
        flops32 = 2 * D + 2 * D + 4
    else:
        ints, fp32, fp64, trans = rng + D, 0.0, 2.0 * D, 0.0   # shift|1, cvt, fma per coordinate
        fp64 += D + 30 + 1                                       # sum, FP64 sin/exp, accumulation
        flops32 = 0
    total = ints + fp32 + fp64 + trans
    return dict(rng=rng, int=ints, fp32=fp32, fp64=fp64, trans=trans, total=total, fp32_flops=flops32)


def alu_roofline(samples_per_s: float, integrand: str, D: int, eval_: str) -> dict:
    """Issue roofline: a CU issues at most 128 VALU lane-instructions per
    clock, so samples/s <= 7.86e13 / instructions per sample.  Also the
    integer-issue view: integer and FP64 instructions issue at about 64
    lanes per CU per clock (no dual issue among them; measured 52-66)."""
    n = valu_instructions_per_sample(integrand, D, eval_)
    achieved = samples_per_s * n["total"]
    int_rate = samples_per_s * (n["int"] + n["fp64"])
    return dict(achieved=achieved, peak=VALU_PEAK, frac=achieved / VALU_PEAK, instructions_per_sample=n,
                roofline_samples_per_s=VALU_PEAK / n["total"],
                int_issue_frac=int_rate / (N_CU * CLOCK_HZ * INT_LANES_PER_CU_CLK),
                int_bound_samples_per_s=N_CU * CLOCK_HZ * INT_LANES_PER_CU_CLK / (n["int"] + n["fp64"]))


WORKLOADS = {
    "sin6d": ("sin6d", "sin_sum", "f1 = sin(sum x_i) on [0,10]^6, d=6 (46656 root cubes), N=16384, n1=5, "
              "max_depth=2, sigma_mult=1, seed=1"),
    "gauss9d": ("narrow_gauss9d", "gauss", "prod exp(-(x_i-0.5)^2/(2*0.02^2)) on [0,1]^9, d=3 (19683 cubes), "
                "N=65536, n1=5, max_depth=3, sigma_mult=0.5, seed=1"),
    "gauss4d": ("gauss4d", "gauss", "exp(-|x|^2/(2*0.2^2)) on [-1,1]^4, d=4 (256 cubes), N=4096, n1=5, "
                "max_depth=1, sigma_mult=1, seed=1"),
}


# The files the sampling kernel's code comes from, with the build flags (the
# level kernels' arguments and launchers in zmc_kernels.hpp do not enter it).
KERNEL_SOURCES = ("paper_1902_07916_amd/build.py", "paper_1902_07916_amd/csrc/zmc_sample.hip",
                  "paper_1902_07916_amd/csrc/zmc_sample_core.hpp", "paper_1902_07916_amd/csrc/zmc_integrands.hpp",
                  "paper_1902_07916_amd/csrc/zmc_device.hpp")
TUNE_TABLE = "paper_1902_07916_amd/csrc/zmc_tune_gfx950.json"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sample_kernel.json")
ISSUE_FILE = os.path.join(ROOT, "profiles", "issue_sample_kernel.json")


def kernel_source_hash(bucket: str) -> str:
    """Hash of what decides one sampling bucket's machine code and launch:
    the kernel sources and the tuning table's entries for that bucket
    ("integrand:dim:eval")."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, TUNE_TABLE)) as fh:
        table = json.load(fh)
    h.update(json.dumps({k: v for k, v in sorted(table.items()) if k.startswith(bucket + ":")}).encode())
    return h.hexdigest()[:16]


def workload_bucket(workload: str) -> str:
    """The (integrand, dim, eval) bucket of a workload's FP32 sampling kernel."""
    from paper_1902_07916_amd import INTEGRANDS, workloads
    gen, integrand, _ = WORKLOADS[workload]
    w = getattr(workloads, gen)(eval="fp32")
    return "%d:%d:1" % (INTEGRANDS[integrand], len(w["lower"]))


def measured_traffic(workload: str):
    """HBM bytes per launch of the sampling kernel from the committed
    FETCH_SIZE / WRITE_SIZE runs, or None when the kernel sources or the
    bucket's tuning entries changed since those counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(workload)
    if not e or e.get("source_hash") != kernel_source_hash(workload_bucket(workload)):
        return None
    return e["bytes_per_launch"]


def measured_issue(workload: str):
    """The sampling kernel's measured VALU issue utilisation from the
    committed rocprofv3 counter run (SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU2,
    GRBM_GUI_ACTIVE): the fraction of SIMD quad-cycles issuing at least one
    VALU instruction, of those issuing two, and instructions per quad-cycle;
    None when the kernel sources or the bucket's tuning entries changed
    since."""
    try:
        with open(ISSUE_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(workload)
    if not e or e.get("source_hash") != kernel_source_hash(workload_bucket(workload)):
        return None
    return {k: e[k] for k in ("valu_busy", "dual_issue", "valu_per_quad_cycle")}


def _oracle_problem(w: dict):
    import oracle
    return oracle.problem(w["integrand"], len(w["lower"]), w["lower"], w["upper"], w["divisions"], w["samples"],
                          w["trials"], w["max_depth"], w["sigma_mult"], w["seed"], params=w["params"],
                          rtol=w.get("rtol", 0.0), max_cubes_per_level=w.get("max_cubes_per_level", 0) or (1 << 24),
                          split=w.get("split", 0) or 2)


def _oracle_cubes(args):
    """Worker of the all-core leg: oracle.cube on root cubes first, first +
    stride, ... until `seconds` elapse; returns (cubes, seconds)."""
    w, first, stride, seconds = args
    import oracle
    p = _oracle_problem(w)
    t0 = time.perf_counter()
    n = 0
    c = first
    while time.perf_counter() - t0 < seconds:
        oracle.cube(p, 0, c)
        c += stride
        n += 1
    return n, time.perf_counter() - t0


def _oracle_cube_range(args):
    """Worker of the all-core reduced-size leg: oracle.cube on level-0 cubes
    first, first + stride, ... below n; returns (cubes, seconds)."""
    w, first, stride, n = args
    import oracle
    p = _oracle_problem(w)
    t0 = time.perf_counter()
    k = 0
    for c in range(first, n, stride):
        oracle.cube(p, 0, c)
        k += 1
    return k, time.perf_counter() - t0


def _oracle_whole(w):
    """Worker of the batch-subset leg: one integral's whole tree with the
    oracle; returns (samples, integral, seconds)."""
    import oracle
    t0 = time.perf_counter()
    o = oracle.integrate(_oracle_problem(w))
    return o.n_samples, o.integral, time.perf_counter() - t0


def _oracle_whole_i(args):
    i, w = args
    return i, _oracle_whole(w)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    """Cores this process may use, capped at 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(w: dict, seconds: float, small: dict | None = None) -> dict:
    """The CPU oracle as it stands (plain single-thread FP64 C), timed on this
    host: single thread on the first root cubes of the same workload (all
    trials, all points) until `seconds` elapse; the same per-cube work spread
    over the host's cores by a process pool (cube c to worker c mod P); and,
    if given, the whole tree of a small workload in one thread."""
    import multiprocessing as mp

    import oracle
    oracle.build()
    p = _oracle_problem(w)
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds:
        oracle.cube(p, 0, n)
        n += 1
    dt = time.perf_counter() - t0
    samples = n * w["trials"] * w["samples"]
    out = {"value": samples / dt, "unit": "samples/s", "cores": 1, "kind": "oracle",
           "sample": "level-0 cubes 0..%d of the same workload, %d trials x %d points each (%.3g samples, %.1f s)"
                     % (n - 1, w["trials"], w["samples"], samples, dt),
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    P = host_cores()
    with mp.get_context("spawn").Pool(P) as pool:
        res = pool.map(_oracle_cubes, [(w, i, P, seconds) for i in range(P)])
    n_all = sum(r[0] for r in res)
    t_all = max(r[1] for r in res)
    out["all_cores"] = {"value": n_all * w["trials"] * w["samples"] / t_all, "unit": "samples/s", "cores": P,
                        "sample": "level-0 cubes of the same workload, cube c on worker c mod %d, %.1f s" % (P, t_all)}
    if small is not None:
        ps = _oracle_problem(small)
        t0 = time.perf_counter()
        o = oracle.integrate(ps)
        dt = time.perf_counter() - t0
        out["small_whole_tree"] = {"value": o.n_samples / dt, "unit": "samples/s", "cores": 1, "s": dt,
                                   "samples": o.n_samples, "integral": o.integral,
                                   "sample": "the whole tree of the 4-D Gaussian workload (256 roots, 4096 points, "
                                             "5 trials, one refinement) in one thread"}
    return out


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q
    f = int(math.floor(k))
    c = min(f + 1, len(xs) - 1)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


def run_cpu(a) -> dict:
    """The oracle at reduced sizes on this host, each beside the GPU doing the
    same work: the 4-D Gaussian workload whole, the narrow 9-D Gaussian
    whole at N/16 (both single thread), level 0 of the 6-D sine at N/16 on
    all cores (cube c to worker c mod P), and every 16th integral of the
    Genz batch, whole trees at N/16, on all cores (one integral per task).
    Takes a few minutes."""
    import multiprocessing as mp

    import torch

    import oracle
    from paper_1902_07916_amd import Integrator, request_from_dict, workloads
    oracle.build()
    zi = Integrator(arena_bytes=int(a.arena_gib * (1 << 30)), max_slots=1024)

    def gpu_time(w, reps=3):
        zi.integrate(**w)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = zi.integrate(**w)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, r

    out = {"cpu_model": cpu_model(), "nproc": os.cpu_count()}
    g9 = dict(workloads.narrow_gauss9d(eval="fp64"))
    g9["samples"] //= 16
    for name, w in (("gauss4d_whole", workloads.gauss4d(eval="fp64")), ("narrow_gauss9d_n16_whole", g9)):
        t0 = time.perf_counter()
        o = oracle.integrate(_oracle_problem(w))
        cpu_s = time.perf_counter() - t0
        row = {"cores": 1, "cpu_s": cpu_s, "samples": o.n_samples, "cpu_samples_per_s": o.n_samples / cpu_s,
               "cpu_integral": o.integral, "cpu_levels": [L.n for L in o.levels]}
        for ev in ("fp64", "fp32"):
            dt, r = gpu_time(dict(w, eval=ev))
            row["gpu_%s_s" % ev] = dt
            row["gpu_%s_integral" % ev] = r.integral
            row["gpu_%s_levels" % ev] = r.cubes_per_level[:r.levels_run]
        row["speedup_gpu_fp32"] = cpu_s / row["gpu_fp32_s"]
        out[name] = row
        print("%s: cpu %.2f s, gpu fp64 %.4f s, fp32 %.4f s" % (name, cpu_s, row["gpu_fp64_s"], row["gpu_fp32_s"]),
              file=sys.stderr, flush=True)
    w6 = dict(workloads.sin6d(eval="fp64"))
    w6["samples"] //= 16
    w6["max_depth"] = 0
    n = w6["divisions"] ** len(w6["lower"])
    P = host_cores()
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(P) as pool:
        res = pool.map(_oracle_cube_range, [(w6, i, P, n) for i in range(P)])
    cpu_s = time.perf_counter() - t0
    assert sum(k for k, _ in res) == n
    samples = n * w6["trials"] * w6["samples"]
    row = {"cores": P, "cpu_s": cpu_s, "samples": samples, "cpu_samples_per_s": samples / cpu_s}
    for ev in ("fp64", "fp32"):
        row["gpu_%s_s" % ev] = gpu_time(dict(w6, eval=ev))[0]
    row["speedup_gpu_fp32"] = cpu_s / row["gpu_fp32_s"]
    out["sin6d_n16_level0_all_cores"] = row
    # every 16th integral of the batch at N/16: integrals are independent, so
    # a subset's results do not depend on the rest of the batch
    sub = workloads.genz_batch(n=a.batch_n, max_cubes_per_level=a.batch_cap, samples=4096 // 16)[::16]
    t0 = time.perf_counter()
    res = [None] * len(sub)
    with mp.get_context("spawn").Pool(P) as pool:
        for k, (i, r) in enumerate(pool.imap_unordered(_oracle_whole_i, list(enumerate(sub)))):
            res[i] = r
            if k % 32 == 31:
                print("batch subset: %d of %d integrals done on the CPU, %.0f s" % (
                    k + 1, len(sub), time.perf_counter() - t0), file=sys.stderr, flush=True)
    cpu_s = time.perf_counter() - t0
    samples = sum(r[0] for r in res)
    row = {"cores": P, "integrals": len(sub), "cpu_s": cpu_s, "samples": samples,
           "cpu_samples_per_s": samples / cpu_s, "cpu_integrals_per_s": len(sub) / cpu_s,
           "cpu_task_s_max": max(r[2] for r in res)}
    for ev in ("fp64", "fp32"):
        reqs = [request_from_dict(dict(w, eval=ev)) for w in sub]
        zi.integrate_batch(reqs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = zi.integrate_batch(reqs)
        torch.cuda.synchronize()
        row["gpu_%s_s" % ev] = time.perf_counter() - t0
        row["gpu_%s_samples" % ev] = sum(o.n_samples for o in outs)
        row["gpu_%s_max_rel_diff" % ev] = max(abs(o.integral - r[1]) / max(abs(r[1]), 1e-300)
                                               for o, r in zip(outs, res))
    row["speedup_gpu_fp32"] = cpu_s / row["gpu_fp32_s"]
    out["genz_batch_every16th_n16_all_cores"] = row
    print("batch subset: cpu %.1f s on %d cores, gpu fp32 %.4f s" % (cpu_s, P, row["gpu_fp32_s"]),
          file=sys.stderr, flush=True)
    zi.close()
    return out


def run_batch(a, steps=None, warmup=None) -> dict:
    """Batched workload: n independent Genz integrals (D in 2..12) per step,
    all levels of all of them in shared launches."""
    import torch
    from paper_1902_07916_amd import INTEGRANDS, Integrator, request_from_dict, workloads
    steps = a.steps if steps is None else steps
    warmup = a.warmup if warmup is None else warmup
    ws = workloads.genz_batch(n=a.batch_n, max_cubes_per_level=a.batch_cap)
    reqs = [request_from_dict(w) for w in ws]
    zi = Integrator(arena_bytes=int(a.arena_gib * (1 << 30)), max_slots=max(8192, len(reqs)))
    for _ in range(warmup):
        zi.integrate_batch(reqs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [zi.integrate_batch(reqs) for _ in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    zi.close()
    a_steps = steps
    last = outs[-1]
    samples = sum(r.n_samples for o in outs for r in o)
    # minimal VALU instructions of the last step: every sample of every level
    names = {v: k for k, v in INTEGRANDS.items()}
    instr = 0.0
    int_instr = 0.0
    for w, r in zip(ws, last):
        n = valu_instructions_per_sample(names[w["integrand"]], len(w["lower"]), w["eval"])
        pts = sum(int(c) for c in r.cubes_per_level[:r.levels_run]) * w["trials"] * w["samples"]
        instr += n["total"] * pts
        int_instr += (n["int"] + n["fp64"]) * pts
    # sampling-kernel time of the last step: integrals stepped together
    # share one launch set per level, whose HIP-event time every one of them
    # records; count each (level, time) once
    k_ms = sum(ms for _, ms in {(l, float(r.sample_ms_per_level[l])) for r in last for l in range(r.levels_run)})
    return {"integrals_per_s": len(reqs) * a_steps / dt, "samples_per_s": samples / dt,
            "ms_per_step": dt * 1e3 / a_steps, "steps": a_steps, "warmup": warmup, "n_integrals": len(reqs),
            "status_ok": sum(r.status == 0 for r in last), "truncated": sum(bool(r.flags & 1) for r in last),
            "fp32_range": sum(bool(r.flags & 4) for r in last),
            "cubes_total": sum(r.n_cubes for r in last), "samples_per_step": samples // a_steps,
            "sample_kernel_ms_per_step": k_ms,
            "alu_frac_sampling": instr / (k_ms * 1e-3) / VALU_PEAK if k_ms > 0 else None,
            "int_issue_frac_sampling": (int_instr / (k_ms * 1e-3) / (N_CU * CLOCK_HZ * INT_LANES_PER_CU_CLK)
                                        if k_ms > 0 else None),
            "alu_frac_wall": instr / (dt / a_steps) / VALU_PEAK}


def run_serve(a, duration=None) -> dict:
    """Serving workload: a Poisson stream of requests submitted in real time;
    latency = submit -> result visible to poll."""
    from paper_1902_07916_amd import Integrator, request_from_dict, workloads
    duration = a.duration if duration is None else duration
    stream = workloads.serving_stream(rate=a.rate, duration=duration)
    reqs = [request_from_dict(w) for _, w in stream]
    zi = Integrator(arena_bytes=int(a.arena_gib * (1 << 30)), serve=True)
    # warm the kernels of every (integrand, D) bucket once; then the cost of
    # a level beyond its sampling launches: the first 200 requests run
    # alone, wall time per level minus the sampling launches' HIP-event time
    for rq in reqs[:64]:
        zi.integrate_request(rq)
    over = []
    for rq in reqs[:200]:
        r = zi.integrate_request(rq)
        over += [m - s for m, s in zip(r.ms_per_level, r.sample_ms_per_level)]
    t0 = time.perf_counter()
    tickets = []
    for (t, _), rq in zip(stream, reqs):
        while True:
            now = time.perf_counter() - t0
            if now >= t:
                break
            time.sleep(min(0.001, t - now))
        tickets.append(zi.submit(rq))
    res = [zi.poll(tk, wait=True) for tk in tickets]
    dt = time.perf_counter() - t0
    st = zi.serve_stats()
    lat = [r.latency_ms for r in res]
    # p99 latency in the stream by the request's own work: its engine time
    # when it runs alone afterwards (same lane arena, nothing beside it)
    own = []
    for rq in reqs:
        own.append(sum(zi.integrate_request(rq).ms_per_level))
    zi.close()
    by_own = {}
    for name, lo, hi in (("own<0.2ms", 0.0, 0.2), ("0.2-1ms", 0.2, 1.0), ("1-5ms", 1.0, 5.0), ("own>=5ms", 5.0, 1e30)):
        sel = [x for x, o in zip(lat, own) if lo <= o < hi]
        by_own[name] = {"requests": len(sel), "p99_ms": percentile(sel, 0.99) if sel else None}
    return {"requests": len(res), "offered_rate": a.rate, "duration_s": duration, "wall_s": dt,
            "integrals_per_s": len(res) / dt, "p50_ms": percentile(lat, 0.5), "p99_ms": percentile(lat, 0.99),
            "max_ms": max(lat), "rtol_met": sum(bool(r.flags & 2) for r in res) / len(res),
            "status_ok": sum(r.status == 0 for r in res), "samples": sum(r.n_samples for r in res),
            "samples_per_s": sum(r.n_samples for r in res) / dt, "levels_stepped": st["levels"],
            "level_cost_beyond_sampling_ms": {"p50": percentile(over, 0.5), "p90": percentile(over, 0.9),
                                              "levels": len(over)},
            "p99_by_own_work": by_own}


# The paper's own timings on its hardware (Tables 1-4), seconds per run.
PAPER_TIMES = {"f1_tf": (355.8, "1 x K40m"), "f1_numba": (313.5, "1 x K40m"), "f1_ray": (38.7, "1 x V100"),
               "f2_numba": (69.7, "1 x K40m"), "f2_ray": (4.8, "1 x V100"), "f2_12d_ray": (47.6, "1 x V100")}
# The paper's results for the same runs (Tables 1-4): value, standard deviation.
PAPER_RESULTS = {"f1_tf": (-48.96, 0.76), "f1_numba": (-49.56, 1.40), "f1_ray": (-49.3971, 0.4845),
                 "f2_numba": (1.00001, 0.00051), "f2_ray": (1.00035, 0.00064), "f2_12d_ray": (1.00002, 0.00079)}


def run_paper(a) -> dict:
    """The paper's parameter sets on this GPU, 10 seeds each (the paper
    averages 10 independent runs): mean result, spread, time per run."""
    import statistics

    import torch
    from paper_1902_07916_amd import Integrator, workloads
    zi = Integrator(arena_bytes=int(a.arena_gib * (1 << 30)))
    out = {}
    for name in workloads.PAPER_RUNS:
        row = {"setting": workloads.PAPER_RUNS[name]["ref"], "paper_result": PAPER_RESULTS[name],
               "paper_s_per_run": PAPER_TIMES[name][0], "paper_hw": PAPER_TIMES[name][1]}
        # two readings of the split (bisection of every axis; d parts per
        # axis as at the root) in both evaluation precisions
        for reading, split in (("bisect", 0), ("kway", workloads.PAPER_RUNS[name]["divisions"])):
            for ev in ("fp32", "fp64"):
                zi.integrate(**workloads.paper_run(name, eval=ev, seed=1, split=split))
                torch.cuda.synchronize()
                res, times = [], []
                for seed in range(1, 11):
                    w = workloads.paper_run(name, eval=ev, seed=seed, split=split)
                    t0 = time.perf_counter()
                    r = zi.integrate(**w)
                    times.append(time.perf_counter() - t0)
                    res.append(r)
                vals = [r.integral for r in res]
                key = "%s_%s" % (reading, ev)
                row[key] = {"mean": statistics.mean(vals), "spread": statistics.pstdev(vals),
                            "mean_stderr": statistics.mean(r.stderr for r in res),
                            "s_per_run": statistics.mean(times),
                            "samples_per_run": statistics.mean(r.n_samples for r in res),
                            "samples_per_s": statistics.mean(r.n_samples for r in res) / statistics.mean(times),
                            "levels_seed1": res[0].cubes_per_level[:res[0].levels_run],
                            "values": vals,
                            "levels_per_seed": [r.cubes_per_level[:r.levels_run] for r in res],
                            "truncated": sum(bool(r.flags & 1) for r in res),
                            "fp32_range_flagged": sum(bool(r.flags & 4) for r in res)}
                print("%s %s: mean %.6g spread %.3g, %.4f s/run, levels %s" % (
                    name, key, row[key]["mean"], row[key]["spread"], row[key]["s_per_run"],
                    row[key]["levels_seed1"]), file=sys.stderr, flush=True)
        out[name] = row
    zi.close()
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sin6d", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="single", choices=["single", "batch", "serve", "paper", "cpu"])
    ap.add_argument("--no-fp64", action="store_true", help="skip timing the plain FP64 path")
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--batch-steps", type=int, default=1,
                    help="timed steps of the batched leg in the default run (0 = skip)")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="length of the serving leg's request stream in the default run (0 = skip)")
    ap.add_argument("--arena-gib", type=float, default=48.0)
    ap.add_argument("--batch-n", type=int, default=4096)
    ap.add_argument("--batch-cap", type=int, default=1 << 20)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--duration", type=float, default=60.0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy a buffer of this size with a plain copy kernel (calibrates HBM byte counters)")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the work would shard by whole "
              "integrals or by contiguous uid ranges with one small all-reduce per level); run with --gpus 1",
              file=sys.stderr)
        return 2

    import torch
    from paper_1902_07916_amd import Integrator, workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    # a plain copy of known size first: the HBM byte counters of a profiled
    # run are calibrated against it
    if a.copy_calibration_mib > 0:
        src = torch.ones(a.copy_calibration_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.mode == "paper":
        print(json.dumps({"mode": "paper", **run_paper(a)}))
        return 0
    if a.mode == "batch":
        print(json.dumps({"mode": "batch", **run_batch(a)}))
        return 0
    if a.mode == "cpu":
        print(json.dumps({"mode": "cpu", **run_cpu(a)}))
        return 0
    if a.mode == "serve":
        print(json.dumps({"mode": "serve", **run_serve(a)}))
        return 0
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
    k_rate = k_samples / (k_ms * 1e-3)
    rl = alu_roofline(k_rate, integrand, D, "fp32")
    roofline = {"bound": "alu", "achieved": rl["achieved"], "peak": VALU_PEAK, "unit": "VALU lane-instructions/s",
                "frac": rl["frac"], "traffic": measured_traffic(a.workload),
                "kernel": "sample_kernel<%s,D=%d,FP32>" % (integrand, D),
                "avg_launch_ms": k_ms / max(k_launches, 1), "launches": k_launches,
                "instructions_per_sample": rl["instructions_per_sample"], "kernel_samples_per_s": k_rate,
                "roofline_samples_per_s": rl["roofline_samples_per_s"],
                "int_issue_frac": rl["int_issue_frac"], "int_bound_samples_per_s": rl["int_bound_samples_per_s"],
                "fp32_flop_frac": k_rate * rl["instructions_per_sample"]["fp32_flops"] / FP32_PEAK_FLOPS,
                "measured_issue": measured_issue(a.workload)}

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
        # the plain FP64 path, warmed and timed exactly like the FP32 one
        for _ in range(a.warmup):
            zi.integrate(**w64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res64 = [zi.integrate(**w64) for _ in range(a.steps)]
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t0
        r64 = res64[-1]
        v64 = sum(x.n_samples for x in res64) / dt64
        k64 = sum(sum(x.sample_ms_per_level) for x in res64)
        out["fp64_path"] = {"value": v64, "unit": "samples/s", "ms_per_step": dt64 * 1e3 / a.steps,
                            "steps": a.steps, "warmup": a.warmup,
                            "kernel_samples_per_s": sum(x.n_samples for x in res64) / (k64 * 1e-3),
                            "integral": r64.integral, "stderr": r64.stderr, "levels": r64.cubes_per_level,
                            "speedup_fp32_over_fp64": value / v64,
                            "rel_diff_fp32_vs_fp64": abs(r.integral - r64.integral) / abs(r64.integral)}
    zi.close()
    if a.batch_steps > 0:
        print("bench: batched leg", file=sys.stderr, flush=True)
        out["batch"] = {"workload": "4096 Genz integrals, D in 2..12, N=4096, n1=3, max_depth=2, sigma_mult=5, "
                                    "seed=7, level cap 2^20, FP32 evaluation", **run_batch(a, a.batch_steps, 1)}
    if a.serve_seconds > 0:
        print("bench: serving leg", file=sys.stderr, flush=True)
        out["serving"] = {"workload": "Poisson %.0f requests/s for %.0f s, Genz integrals D in 3..12, rtol "
                                      "10^U(-5,-3), seed=11" % (a.rate, a.serve_seconds),
                          **run_serve(a, a.serve_seconds)}
    if a.cpu_seconds > 0:
        print("bench: CPU oracle leg", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w64, a.cpu_seconds, small=workloads.gauss4d(eval="fp64"))
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
