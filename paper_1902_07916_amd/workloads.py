"""Seeded synthetic workloads (inputs only; no arithmetic of the method).

Shared by the tests (for both the HIP path and the oracle), the benchmark and
the smoke check.  Every workload is a plain dict of request fields:
integrand, params, lower, upper, divisions, samples, trials, max_depth,
sigma_mult, seed, eval [, rtol, max_cubes_per_level].

The analytic integrands need no dataset.  The paper's own tests (Sec. 3) are
f1 = sin(sum x_i) on [0,10]^6 and a normalised 9-D Gaussian on [-1,1]^9; the
batched and serving workloads draw Genz-family integrands (oscillatory,
product peak, corner peak, Gaussian) with random coefficients.
"""
from __future__ import annotations

import math

import numpy as np

GAUSS, SIN_SUM, GENZ_OSC, GENZ_PPEAK, GENZ_CPEAK, GENZ_GAUSS, CONST, MONOMIAL = range(8)
GENZ_FAMILIES = (GENZ_OSC, GENZ_PPEAK, GENZ_CPEAK, GENZ_GAUSS)


def gauss4d(eval="fp64", samples=4096):
    """4-D Gaussian exp(-|x|^2 / (2 * 0.2^2)) on [-1,1]^4, 4 divisions per axis
    (256 cubes), 4096 points per cube, 5 trials, one refinement, sigma 1."""
    return dict(integrand=GAUSS, params=[0.2, 1.0, 0.0, 0.0, 0.0, 0.0], lower=[-1.0] * 4, upper=[1.0] * 4,
                divisions=4, samples=samples, trials=5, max_depth=1, sigma_mult=1.0, seed=1, eval=eval)


def sin6d(eval="fp32", samples=16384, divisions=6, max_depth=2):
    """The paper's f1 = sin(sum_{i=1..6} x_i) on [0,10]^6: 6 divisions per axis
    (46656 cubes), 16384 points per cube, 5 trials, two refinements, sigma 1."""
    return dict(integrand=SIN_SUM, params=[], lower=[0.0] * 6, upper=[10.0] * 6, divisions=divisions,
                samples=samples, trials=5, max_depth=max_depth, sigma_mult=1.0, seed=1, eval=eval)


def narrow_gauss9d(eval="fp32", samples=65536, max_depth=3):
    """Narrow 9-D Gaussian prod exp(-(x_i-0.5)^2 / (2 * 0.02^2)) on [0,1]^9:
    3 divisions per axis (19683 cubes), 65536 points per cube, 5 trials,
    three refinements, sigma 0.5 (a very uneven tree)."""
    return dict(integrand=GAUSS, params=[0.02, 1.0] + [0.5] * 9, lower=[0.0] * 9, upper=[1.0] * 9, divisions=3,
                samples=samples, trials=5, max_depth=max_depth, sigma_mult=0.5, seed=1, eval=eval)


def paper_f2(sigma=0.01, dim=9, divisions=3, samples=3**9, trials=5, max_depth=3, sigma_mult=5.0,
             eval="fp32", seed=1):
    """The paper's normalised f2 = (sqrt(2 pi) sigma)^-D exp(-|x|^2 / (2 sigma^2))
    on [-1,1]^D (Sec. 3; Table 2 parameters by default: 3 sub-domains per
    axis, 3^9 points per sub-domain, 5 trials, partition depth 4, 5 sigma)."""
    A = (math.sqrt(2 * math.pi) * sigma) ** -dim
    return dict(integrand=GAUSS, params=[sigma, A] + [0.0] * dim, lower=[-1.0] * dim, upper=[1.0] * dim,
                divisions=divisions, samples=samples, trials=trials, max_depth=max_depth,
                sigma_mult=sigma_mult, seed=seed, eval=eval)


# The paper's own runs (Sec. 3), with its "partition depth" p mapped to
# max_depth = p - 1 and a k-sigma cut to sigma_mult = k.  Points per
# sub-domain are n2^D where the paper gives points per dimension.
PAPER_RUNS = {
    # f1 = sin(sum x), [0,10]^6
    "f1_tf": dict(f="f1", divisions=3, samples=20 ** 6, max_depth=1, sigma_mult=5.0,
                  ref="TensorFlow version, Table 1: 3 sub-domains/axis, 20 points/axis, 5 trials, depth 2, 5 sigma"),
    "f1_numba": dict(f="f1", divisions=6, samples=10 ** 6, max_depth=1, sigma_mult=5.0,
                     ref="Numba multiprocessing version, Table 1: 6/axis, 10 points/axis, 5 trials, depth 2, 5 sigma"),
    "f1_ray": dict(f="f1", divisions=12, samples=10 ** 4, max_depth=0, sigma_mult=5.0,
                   ref="Numba-Ray version, Table 3: 12/axis, 1e4 points, 5 trials, depth 1"),
    # normalised f2, sigma = 0.01, [-1,1]^9
    "f2_numba": dict(f="f2", divisions=3, samples=3 ** 9, max_depth=3, sigma_mult=5.0,
                     ref="Numba multiprocessing version, Table 2: 3/axis, 3 points/axis, 5 trials, depth 4, 5 sigma"),
    "f2_ray": dict(f="f2", divisions=3, samples=10 ** 4, max_depth=3, sigma_mult=4.0,
                   ref="Numba-Ray version, Table 4: 3/axis, 1e4 points, 5 trials, depth 4, 4 sigma"),
    # the 12-D Gaussian of Table 4, at the 9-D run's parameters (the paper
    # gives none of its own); with 3 parts per axis its depth-4 tree names
    # 3^48 ~ 2^76 sub-domains, which takes cube ids past 64 bits
    "f2_12d_ray": dict(f="f2", dim=12, divisions=3, samples=10 ** 4, max_depth=3, sigma_mult=4.0,
                       ref="Numba-Ray version, Table 4, 12-D: 3/axis, 1e4 points, 5 trials, depth 4, 4 sigma"),
}


def paper_run(name, eval="fp32", seed=1, split=0):
    """One of the paper's parameter sets (see PAPER_RUNS).  split = 0
    bisects every axis of a selected cube; split = r["divisions"] is the
    literal reading of Sec. 2.1 (a selected cube is cut into as many equal
    parts as the domain was, d per axis)."""
    r = PAPER_RUNS[name]
    if r["f"] == "f1":
        w = sin6d(eval=eval, samples=r["samples"], divisions=r["divisions"], max_depth=r["max_depth"])
        w["sigma_mult"] = r["sigma_mult"]
    else:
        w = paper_f2(dim=r.get("dim", 9), divisions=r["divisions"], samples=r["samples"],
                     max_depth=r["max_depth"], sigma_mult=r["sigma_mult"], eval=eval)
    w["seed"] = seed
    w["split"] = split
    return w


def _genz_params(fam, rng, D):
    c = rng.uniform(0.5, 5.0, D)
    w = rng.uniform(0.0, 1.0, D)
    u = rng.uniform()
    if fam == GENZ_OSC:
        return [u] + c.tolist()
    if fam == GENZ_PPEAK:
        return c.tolist() + w.tolist()
    if fam == GENZ_CPEAK:
        return c.tolist()
    return c.tolist() + w.tolist()


def _seeds(master, n):
    ss = np.random.SeedSequence(master).spawn(n)
    out = []
    for s in ss:
        st = s.generate_state(2, np.uint32)
        out.append(int(st[0]) | (int(st[1]) << 32))
    return out


def genz_batch(n=4096, seed=7, samples=4096, trials=3, max_depth=2, sigma_mult=5.0, eval="fp32",
               max_cubes_per_level=0, max_root_cubes=100_000):
    """Batched workload: n independent Genz integrals on [0,1]^D with D uniform
    in 2..12, family uniform over {osc, ppeak, cpeak, gauss}, c_i ~ U(0.5, 5),
    w_i ~ U(0, 1), u ~ U(0, 1), divisions d ~ U{2..6} reduced while d^D
    exceeds max_root_cubes.  Draw order per integral: D, family, c, w, u, d.
    Per-integral RNG keys from SeedSequence(seed).spawn(n)."""
    rng = np.random.default_rng(seed)
    keys = _seeds(seed, n)
    out = []
    for i in range(n):
        D = int(rng.integers(2, 13))
        fam = GENZ_FAMILIES[int(rng.integers(0, 4))]
        params = _genz_params(fam, rng, D)
        d = int(rng.integers(2, 7))
        while d ** D > max_root_cubes and d > 1:
            d -= 1
        out.append(dict(integrand=fam, params=params, lower=[0.0] * D, upper=[1.0] * D, divisions=d,
                        samples=samples, trials=trials, max_depth=max_depth, sigma_mult=sigma_mult,
                        seed=keys[i], eval=eval, max_cubes_per_level=max_cubes_per_level))
    return out


def serving_stream(rate=200.0, duration=60.0, seed=11, samples=4096, trials=3, max_depth=4, sigma_mult=5.0,
                   eval="fp32", max_root_cubes=4096, max_cubes_per_level=1 << 18):
    """Serving workload: Poisson arrivals at `rate` per second for `duration`
    seconds; each request a Genz integral on [0,1]^D, D uniform in 3..12,
    relative tolerance 10^U(-5,-3), d = the largest of 2..6 with d^D <=
    max_root_cubes.  Returns a list of (arrival_time_s, request dict)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        D = int(rng.integers(3, 13))
        fam = GENZ_FAMILIES[int(rng.integers(0, 4))]
        params = _genz_params(fam, rng, D)
        rtol = 10.0 ** rng.uniform(-5.0, -3.0)
        d = max([1] + [dd for dd in range(2, 7) if dd ** D <= max_root_cubes])
        out.append((t, dict(integrand=fam, params=params, lower=[0.0] * D, upper=[1.0] * D, divisions=d,
                            samples=samples, trials=trials, max_depth=max_depth, sigma_mult=sigma_mult,
                            seed=0, eval=eval, rtol=rtol, max_cubes_per_level=max_cubes_per_level)))
    keys = _seeds(seed, len(out))
    for (_, r), k in zip(out, keys):
        r["seed"] = k
    return out
