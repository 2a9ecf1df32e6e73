"""Autotuner for the sampling kernel's tile shape.

    python -m paper_1902_07916_amd.tune --out tune.json [--dims 2-12] [--integrands genz_osc,...]
    python -m paper_1902_07916_amd.tune --waves --out tune.json --dims 1-16 --evals fp32,fp64
    python -m paper_1902_07916_amd.tune --blocks --out tune.json --dims 1-16 --samples 4096

For every (integrand, D, eval) bucket it times the sampling launches of one
level over the root cubes of [0,1]^D (N points per cube, 16384 unless
--samples, 3 trials; HIP events on the launch stream, the fastest of 5 runs)
for each candidate cap on the 4-point groups a thread takes per chunk (the
chunk is 4 * 64 * groups points per wave), and writes the fastest as a
JSON object {"integrand:dim:eval": groups, ...} that zmc_init() reads from
`tune_path`.  --waves picks each bucket's occupancy variant and --blocks its
block shape (threads per sampling block) by timing the sampling launches.  The table depends only on the bucket, never on what else is
resident, so a request's result stays independent of its batch.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

CANDIDATES = (2, 4, 8, 16, 32)


def _parse_dims(s: str):
    if "-" in s:
        a, b = s.split("-")
        return list(range(int(a), int(b) + 1))
    return [int(v) for v in s.split(",")]


def _params(name: str, D: int):
    if name == "gauss":
        return [0.3, 1.0] + [0.5] * D
    if name == "sin_sum":
        return []
    if name == "genz_osc":
        return [0.25] + [2.0] * D
    if name in ("genz_ppeak", "genz_gauss"):
        return [2.0] * D + [0.5] * D
    if name == "genz_cpeak":
        return [1.0] * D
    raise ValueError(name)


def time_bucket(name: str, D: int, eval_: str, groups: int, n_cubes: int = 4096, reps: int = 5,
                N: int = 16384) -> float:
    """Seconds per sample of the sampling launches with the given cap: one
    level over d^D >= n_cubes root cubes (3 trials), the launches' HIP-event
    time, the fastest of `reps` runs after a warm-up run."""
    import torch
    from paper_1902_07916_amd import INTEGRANDS, Integrator, make_request
    key = "%d:%d:%d" % (INTEGRANDS[name], D, 1 if eval_ == "fp32" else 0)
    with tempfile.NamedTemporaryFile("w", suffix=".json", delete=False) as fh:
        json.dump({key: groups}, fh)
        path = fh.name
    try:
        zi = Integrator(arena_bytes=2 << 30, tune_path=path)
        d = 2
        while d ** D < n_cubes and d < 64:
            d += 1
        req = make_request(name, _params(name, D), [0.0] * D, [1.0] * D, d, N, 3, 0, 1.0, 1, eval=eval_)
        zi.integrate_request(req)
        torch.cuda.synchronize()
        rs = [zi.integrate_request(req) for _ in range(reps)]
        zi.close()
        return min(r.sample_ms_per_level[0] for r in rs) * 1e-3 / rs[0].n_samples
    finally:
        os.unlink(path)


REGISTRY = ("sin_sum", "gauss", "genz_osc", "genz_ppeak", "genz_cpeak", "genz_gauss")
WAVE_HINTS = (1, 5, 7, 8)  # the library's occupancy variants (minimum waves per SIMD)
MIN_GAIN = 1.015        # a variant must beat the unconstrained kernel by 1.5% to be chosen
# Seconds of back-to-back runs of a bucket's level before it is timed: the
# GPU clock rises over the first tens of milliseconds of load, and a short
# level timed from a colder state runs up to 12% slower.
WARM_S = 0.05


def _bucket_rate(zi, name, D, ev, n_target, N, trials):
    """Samples/s of the sampling launches (HIP events, best of 3, after
    WARM_S of warm-up runs) over one level of d^D >= n_target root cubes of
    [0,1]^D."""
    import torch
    from paper_1902_07916_amd import make_request
    d = 2
    while d ** D < n_target:
        d += 1
    req = make_request(name, _params(name, D), [0.0] * D, [1.0] * D, d, N, trials, 0, 1.0, 1, eval=ev)
    t0 = time.perf_counter()
    zi.integrate_request(req)
    while time.perf_counter() - t0 < WARM_S:
        zi.integrate_request(req)
    torch.cuda.synchronize()
    rs = [zi.integrate_request(req) for _ in range(3)]
    ms = min(r.sample_ms_per_level[0] for r in rs)
    return d ** D, rs[0].n_samples / (ms * 1e-3)


def rate_table(evals=("fp32", "fp64"), dims=(2, 4, 6, 9, 12, 16), n_target=65536, N=16384, trials=3,
               tune_path=None, names=None, roots=None):
    """Sampling-kernel rate per bucket from HIP-event kernel time, with the
    fraction of the ALU roofline.  roots: several level sizes (minimum root
    cubes) per bucket instead of n_target alone."""
    from paper_1902_07916_amd import Integrator
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    zi = Integrator(arena_bytes=16 << 30, tune_path=tune_path)
    rows = []
    for ev in evals:
        for name in (names or REGISTRY):
            for D in dims:
                if ev == "fp64" and D not in (4, 6, 9):
                    continue
                for target in (roots or (n_target,)):
                    cubes, sps = _bucket_rate(zi, name, D, ev, target, N, trials)
                    rl = bench.alu_roofline(sps, name, D, ev)
                    rows.append(dict(eval=ev, integrand=name, D=D, cubes=cubes, samples_per_s=sps, frac=rl["frac"],
                                     int_issue_frac=rl["int_issue_frac"]))
                    print("%s %-11s D=%2d cubes=%7d %.3e samples/s  %5.1f%% of the VALU issue roofline, %5.1f%% "
                          "of integer issue" % (ev, name, D, cubes, sps, 100 * rl["frac"], 100 * rl["int_issue_frac"]),
                          flush=True)
    zi.close()
    return rows


def wave_sweep(out_path, evals=("fp32", "fp64"), dims=range(1, 17), n_target=16384, N=16384, trials=3):
    """Time every occupancy variant of every registry bucket and write the
    fastest as {"integrand:dim:eval:w": waves} (merged into out_path)."""
    from paper_1902_07916_amd import INTEGRANDS, Integrator
    rates = {}
    for w in WAVE_HINTS:
        table = {"%d:%d:%d:w" % (INTEGRANDS[n], D, 1 if ev == "fp32" else 0): w
                 for n in REGISTRY for D in dims for ev in evals}
        with tempfile.NamedTemporaryFile("w", suffix=".json", delete=False) as fh:
            json.dump(table, fh)
            path = fh.name
        try:
            zi = Integrator(arena_bytes=16 << 30, tune_path=path)
            for ev in evals:
                for name in REGISTRY:
                    for D in dims:
                        rates[(name, D, ev, w)] = _bucket_rate(zi, name, D, ev, n_target, N, trials)[1]
                        print("w%d %s %-11s D=%2d %.3e samples/s" % (w, ev, name, D, rates[(name, D, ev, w)]),
                              flush=True)
            zi.close()
        finally:
            os.unlink(path)
    best = json.load(open(out_path)) if os.path.exists(out_path) else {}
    for ev in evals:
        for name in REGISTRY:
            for D in dims:
                r = {w: rates[(name, D, ev, w)] for w in WAVE_HINTS}
                w_best = max(r, key=r.get)
                if r[w_best] < MIN_GAIN * r[1]:
                    w_best = 1  # within the timing noise: keep the unconstrained kernel
                best["%d:%d:%d:w" % (INTEGRANDS[name], D, 1 if ev == "fp32" else 0)] = w_best
                print("%s %-11s D=%2d  %s  best %d (%.1f%% over 1)" % (
                    ev, name, D, " ".join("w%d:%.3e" % (w, v) for w, v in r.items()), w_best,
                    100 * (r[w_best] / r[1] - 1)), flush=True)
    with open(out_path, "w") as fh:
        json.dump(best, fh, indent=1, sort_keys=True)
    return best


BLOCKS = (64, 128, 256)  # threads per sampling block


def block_sweep(out_path, evals=("fp32",), dims=range(1, 17), n_target=65536, N=4096, trials=3):
    """Time every block shape of every registry bucket (each in its built-in
    occupancy variant) and write the fastest as {"integrand:dim:eval:b":
    threads} (merged into out_path); 256 is kept unless another shape is
    MIN_GAIN faster."""
    from paper_1902_07916_amd import INTEGRANDS, Integrator
    rates = {}
    for b in BLOCKS:
        table = {"%d:%d:%d:b" % (INTEGRANDS[n], D, 1 if ev == "fp32" else 0): b
                 for n in REGISTRY for D in dims for ev in evals}
        with tempfile.NamedTemporaryFile("w", suffix=".json", delete=False) as fh:
            json.dump(table, fh)
            path = fh.name
        try:
            zi = Integrator(arena_bytes=16 << 30, tune_path=path)
            for ev in evals:
                for name in REGISTRY:
                    for D in dims:
                        rates[(name, D, ev, b)] = _bucket_rate(zi, name, D, ev, n_target, N, trials)[1]
                        print("b%d %s %-11s D=%2d %.3e samples/s" % (b, ev, name, D, rates[(name, D, ev, b)]),
                              flush=True)
            zi.close()
        finally:
            os.unlink(path)
    best = json.load(open(out_path)) if os.path.exists(out_path) else {}
    for ev in evals:
        for name in REGISTRY:
            for D in dims:
                r = {b: rates[(name, D, ev, b)] for b in BLOCKS}
                b_best = max(r, key=r.get)
                if r[b_best] < MIN_GAIN * r[256]:
                    b_best = 256
                key = "%d:%d:%d:b" % (INTEGRANDS[name], D, 1 if ev == "fp32" else 0)
                if b_best == 256:
                    best.pop(key, None)
                else:
                    best[key] = b_best
                print("%s %-11s D=%2d  %s  best %d (%.1f%% over 256)" % (
                    ev, name, D, " ".join("b%d:%.3e" % (b, v) for b, v in r.items()), b_best,
                    100 * (r[b_best] / r[256] - 1)), flush=True)
    with open(out_path, "w") as fh:
        json.dump(best, fh, indent=1, sort_keys=True)
    return best


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--table", action="store_true", help="print the sampling rate per bucket and exit")
    ap.add_argument("--dims", default=None, help="default 2-12; with --table 2,4,6,9,12,16")
    ap.add_argument("--integrands", default=None)
    ap.add_argument("--evals", default="fp32")
    ap.add_argument("--samples", type=int, default=16384, help="points per cube")
    ap.add_argument("--waves", action="store_true",
                    help="time every occupancy variant of every registry bucket; write the fastest to --out")
    ap.add_argument("--tune-path", default=None, help="tuning file for --table")
    ap.add_argument("--roots", default=None,
                    help="with --table: comma-separated level sizes (minimum root cubes per level; default 65536)")
    ap.add_argument("--blocks", action="store_true",
                    help="time every block shape (64/128/256 threads) of every registry bucket; write the fastest "
                         "to --out")
    a = ap.parse_args(argv)
    if a.table:
        rate_table(evals=a.evals.split(","), N=a.samples, tune_path=a.tune_path,
                   dims=_parse_dims(a.dims) if a.dims else (2, 4, 6, 9, 12, 16),
                   names=a.integrands.split(",") if a.integrands else None,
                   roots=[int(v) for v in a.roots.split(",")] if a.roots else None)
        return 0
    if a.blocks:
        if not a.out:
            ap.error("--blocks needs --out")
        block_sweep(a.out, evals=a.evals.split(","), dims=_parse_dims(a.dims or "2-12"), N=a.samples)
        return 0
    if a.waves:
        if not a.out:
            ap.error("--waves needs --out")
        wave_sweep(a.out, evals=a.evals.split(","), dims=_parse_dims(a.dims or "2-12"), N=a.samples)
        return 0
    if not a.out:
        ap.error("--out is required unless --table")
    from paper_1902_07916_amd import INTEGRANDS
    table = {}
    if os.path.exists(a.out):
        table = json.load(open(a.out))
    for name in (a.integrands or "genz_osc,genz_ppeak,genz_cpeak,genz_gauss,gauss,sin_sum").split(","):
        for D in _parse_dims(a.dims or "2-12"):
            for ev in a.evals.split(","):
                times = {g: time_bucket(name, D, ev, g, N=a.samples) for g in CANDIDATES}
                best = min(times, key=times.get)
                key = "%d:%d:%d" % (INTEGRANDS[name], D, 1 if ev == "fp32" else 0)
                table[key] = best
                print("%-11s D=%2d %s  best groups=%2d  %s" % (name, D, ev, best,
                      " ".join("%d:%.3gns" % (g, t * 1e9) for g, t in times.items())), flush=True)
                with open(a.out, "w") as fh:
                    json.dump(table, fh, indent=1, sort_keys=True)
    return 0


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    sys.exit(main())
