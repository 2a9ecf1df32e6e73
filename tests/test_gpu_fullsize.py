"""Parity at the full benchmark sizes, where the oracle cannot run the whole
tree: every step is checked on what the oracle can compute one by one or on
properties that hold at any size.

 * sampled cubes of every level: m, s recomputed by the oracle;
 * threshold: the oracle's threshold over the GPU's own list of s;
 * selection: the strict rule s > thr against that threshold (bit-exact
   outside a 1e-12 band, which covers only the threshold's rounding);
 * next list: the children of the selected parents in order;
 * totals: the sum of the accepted means / variances of the trace;
 * the integral against the closed form (statistical) and FP32 vs FP64."""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import closed_forms as cf  # noqa: E402
from common import check_levels_sampled, rel  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zi():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_07916_amd import Integrator
    z = Integrator(arena_bytes=48 << 30)
    yield z
    z.close()


def _check_levels(orc, w, r, n_sample, m_tol, m_floor=0.0):
    """m_floor: absolute slack for values FP32 cannot represent (a cube whose
    FP64 estimate is ~1e-200 reads 0 in FP32)."""
    check_levels_sampled(orc, w, r, n_sample, m_tol, m_floor)


@pytest.mark.parametrize("eval_,tol", [("fp32", 2e-5), ("fp64", 1e-12)])
def test_sin6d_full(zi, orc, eval_, tol):
    from paper_1902_07916_amd import workloads as W
    w = W.sin6d(eval=eval_)
    r = zi.integrate(**w, trace=True, trace_capacity=1 << 23)
    assert r.status == 0 and r.levels_run == 3 and r.flags == 0
    print("sin6d %s: I=%.9g stderr=%.3g levels=%s selected=%s" % (eval_, r.integral, r.stderr, r.cubes_per_level,
                                                                 r.selected_per_level))
    _check_levels(orc, w, r, 12, tol)
    exact = cf.f1_exact()
    assert abs(r.integral - exact) <= 5 * r.stderr


def _accepted(L, last):
    keep = np.ones(L["n"], bool) if last else ~L["sel"].astype(bool)
    return L["uid"][keep], L["m"][keep]


def test_sin6d_fp32_vs_fp64(zi):
    """FP32 evaluation against the FP64 path on the same points.  The
    difference splits into (i) arithmetic: cubes evaluated and accepted in
    both runs, and (ii) decisions that flipped within rounding of the
    threshold, after which the two trees estimate that cube differently.
    (i) must be within 1e-4 of |I|; (ii) only at cubes whose FP64 margin is
    below 1e-4."""
    from paper_1902_07916_amd import workloads as W
    a = zi.integrate(**W.sin6d(eval="fp32"), trace=True, trace_capacity=1 << 23)
    b = zi.integrate(**W.sin6d(eval="fp64"), trace=True, trace_capacity=1 << 23)
    arith = 0.0
    flips = 0
    nl = min(a.levels_run, b.levels_run)
    for l in range(nl):
        La, Lb = a.trace[l], b.trace[l]
        last = l == W.sin6d()["max_depth"]
        common, ia, ib = np.intersect1d(La["uid"], Lb["uid"], assume_unique=True, return_indices=True)
        V = (10.0 / 6 / 2**l) ** 6
        assert np.max(np.abs(La["m"][ia] - Lb["m"][ib])) <= 2e-6 * V
        if not last:
            fl = La["sel"][ia] != Lb["sel"][ib]
            flips += int(fl.sum())
            margin = np.abs(Lb["s"][ib] - b.thr_per_level[l]) / b.thr_per_level[l]
            assert np.all(margin[fl] < 1e-4), margin[fl]
            both = ~La["sel"][ia].astype(bool) & ~Lb["sel"][ib].astype(bool)
        else:
            both = np.ones(len(ia), bool)
        arith += float(np.sum(La["m"][ia][both] - Lb["m"][ib][both]))
    total = a.integral - b.integral
    print("fp32-fp64: total %.3g, arithmetic %.3g (%.2g of |I|), flips %d" % (total, arith, abs(arith / b.integral),
                                                                            flips))
    assert abs(arith) <= 1e-4 * abs(b.integral)
    if flips == 0:
        assert rel(a.integral, b.integral) < 1e-4


@pytest.mark.parametrize("eval_,tol", [("fp32", 2e-5), ("fp64", 1e-12)])
def test_gauss9d_full(zi, orc, eval_, tol):
    from paper_1902_07916_amd import workloads as W
    w = W.narrow_gauss9d(eval=eval_)
    r = zi.integrate(**w, trace=True, trace_capacity=1 << 22)
    assert r.status == 0
    print("gauss9d %s: I=%.9g stderr=%.3g levels=%s selected=%s" % (eval_, r.integral, r.stderr,
                                                                   r.cubes_per_level, r.selected_per_level))
    _check_levels(orc, w, r, 3, tol, m_floor=1e-30 if eval_ == "fp32" else 0.0)
    # The peak (width 0.02) sits on the common corner of the 512 level-1
    # children and is hit ~0.17 times per trial, so many cubes see no hit in
    # all 5 trials and are accepted with m = s = 0: the method underestimates
    # here (about 0.6 of the exact value) with an optimistic stderr.  The
    # check is only that the estimate is of the right order.
    exact = cf.gauss(0.02, 1.0, [0.5] * 9, [0.0] * 9, [1.0] * 9)
    assert 0.3 * exact < r.integral < 1.5 * exact


def test_gauss4d_full_vs_closed_form(zi):
    from paper_1902_07916_amd import workloads as W
    r = zi.integrate(**W.gauss4d(eval="fp64"))
    exact = cf.gauss(0.2, 1.0, [0.0] * 4, [-1.0] * 4, [1.0] * 4)
    assert abs(r.integral - exact) <= 5 * r.stderr


def test_genz_batch4096_full(zi):
    """The 4096-integral Genz batch exactly as the benchmark runs it (D = 2..12,
    N = 4096, n1 = 3, max_depth 2, sigma 5, level cap 2^20, FP32 evaluation).

    At full size: every result is OK; per level, selections obey Cantelli's
    bound and the next level holds 2^D children per selected cube unless the
    integral was truncated; the sample count is the sum over levels.  On two
    integrals of each family small enough for the oracle: the batch result is
    bitwise the same as the request alone, and the alone run's whole tree
    matches the oracle (replaying in-band decisions) within 1e-4."""
    from common import compare_tree
    from paper_1902_07916_amd import request_from_dict
    from paper_1902_07916_amd import workloads as W
    import oracle as orc
    ws = W.genz_batch(n=4096, max_cubes_per_level=1 << 20)
    z = zi  # 48 GiB arena, 8192 slots: the benchmark's configuration
    print("batch 4096: integrating", flush=True)
    outs = z.integrate_batch([request_from_dict(w) for w in ws])
    for w, r in zip(ws, outs):
        D = len(w["lower"])
        assert r.status == 0
        n = [int(c) for c in r.cubes_per_level[:r.levels_run]]
        sel = [int(c) for c in r.selected_per_level[:r.levels_run]]
        assert n[0] == w["divisions"] ** D
        assert r.n_samples == sum(n) * w["trials"] * w["samples"]
        for l in range(r.levels_run):
            assert sel[l] <= math.floor(n[l] / (1 + w["sigma_mult"] ** 2))
            if l + 1 < r.levels_run:
                assert n[l + 1] == sel[l] * 2 ** D <= w["max_cubes_per_level"]
        if r.flags & 1:
            assert sel[r.levels_run - 1] * 2 ** D > w["max_cubes_per_level"]
    # per family, two integrals the oracle can run in about a second
    # (300..3000 cubes in all), refined ones first
    picks = []
    for fam in W.GENZ_FAMILIES:
        idx = [i for i, w in enumerate(ws) if w["integrand"] == fam and 300 <= outs[i].n_cubes <= 3000]
        idx.sort(key=lambda i: (-outs[i].levels_run, outs[i].n_cubes))
        picks += idx[:2]
    assert len(picks) >= 6
    for i in picks:
        w = ws[i]
        print("batch 4096: integral %d alone (family %d, D=%d, %d cubes)" % (
            i, w["integrand"], len(w["lower"]), outs[i].n_cubes), flush=True)
        ra = z.integrate(**w, trace=True)
        assert ra.integral == outs[i].integral and ra.std == outs[i].std
        compare_tree(orc, w, ra, 1e-4, 1e-4)


def test_paper_f2_split_readings(zi):
    """The paper's 9-D f2 run of Table 4 (sigma 0.01 on [-1,1]^9, 3/axis,
    1e4 points, 5 trials, depth 4, 4 sigma) in FP64 under both readings of
    the split: with d = 3 parts per axis the result is 1 within its standard
    error, as the paper reports; with bisection the peak sits on the common
    corner of every child and the tree recovers only a small fraction."""
    from paper_1902_07916_amd import workloads as W
    for seed in (1, 2):
        rk = zi.integrate(**W.paper_run("f2_ray", eval="fp64", seed=seed, split=3))
        assert rk.status == 0 and rk.levels_run == 4
        assert abs(rk.integral - 1.0) <= max(5 * rk.stderr, 2e-3), (rk.integral, rk.stderr)
        rb = zi.integrate(**W.paper_run("f2_ray", eval="fp64", seed=seed, split=0))
        assert rb.status == 0 and rb.integral < 0.01, rb.integral


def test_fp32_sine_has_no_mean_error(zi):
    """FP32 evaluation of sin(sum x_i) carries no mean error: over the 12^6
    root cubes of [0,10]^6 (3 trials of 256 points each, 2.3e9 points) the
    signed mean of (f32 - f64) on the same points, relative to mean |f|
    = 2/pi, is below 1e-9.  f1's integral is about 1.3e4 times smaller than
    the integral of |f1|, so a mean error of 1e-9 of |f| would already be
    1.3e-5 of the result.  (Each cube's own difference is ~4e-7 of its
    sum: the FP32 rounding of the per-axis phase steps, which is the same
    for every cube of a level and averages out over the cubes' phases.)"""
    from paper_1902_07916_amd import make_request
    d, D, N, n1 = 12, 6, 256, 3
    uids = np.arange(d ** D, dtype=np.uint64)
    sums = []
    for ev in ("fp32", "fp64"):
        rq = make_request("sin_sum", [], [0.0] * D, [10.0] * D, d, N, n1, 2, 1.0, 11, eval=ev)
        sums.append(zi.cube_estimates(rq, 0, uids)[2])
    diff = sums[0] - sums[1]
    n = diff.size * N
    mean_rel = float(np.sum(diff)) / n / (2 / np.pi)
    per_sum = float(np.sqrt(np.mean(diff ** 2))) / N / (2 / np.pi)
    print("FP32 sine: signed mean error %.3g of mean |f| over %.3g points; per-sum rms %.3g" % (mean_rel, n, per_sum))
    assert abs(mean_rel) < 1e-9
    assert per_sum < 2e-6


FP32_BIAS_CASES = [
    # (integrand, params for D = 4, box): positive families, the integral of
    # |f| is the integral of f
    ("gauss", [0.3, 1.7, 0.2, 0.4, 0.6, 0.5], 0.0, 1.0),
    ("genz_ppeak", [2.0, 4.0, 1.0, 3.0, 0.2, 0.7, 0.9, 0.4], 0.0, 1.0),
    ("genz_cpeak", [0.9, 2.0, 3.5, 1.2], 0.0, 1.0),
    ("genz_gauss", [1.0, 3.0, 0.5, 2.0, 0.2, 0.8, 0.5, 0.1], 0.0, 1.0),
    ("monomial", [1.0, 2.0, 3.0, 4.0], 0.5, 1.5),
]


@pytest.mark.parametrize("name,prm,lo,hi", FP32_BIAS_CASES, ids=[c[0] for c in FP32_BIAS_CASES])
def test_fp32_families_have_no_mean_error(zi, name, prm, lo, hi):
    """FP32 evaluation of every positive registry family against FP64 on the
    same 5e7 points (8^4 root cubes of a 4-D box, 3 trials of 4096 points):
    the signed mean of (f32 - f64), relative to the mean of f, is below
    1e-6 -- a systematic error far inside the 1e-4 tolerance of FP32-mode
    results (measured: the FP32 rounding of the per-cube constants and the
    hardware exp2 / rcp; see the design notes)."""
    from paper_1902_07916_amd import make_request
    d, D, N, n1 = 8, 4, 4096, 3
    uids = np.arange(d ** D, dtype=np.uint64)
    sums = []
    for ev in ("fp32", "fp64"):
        rq = make_request(name, prm, [lo] * D, [hi] * D, d, N, n1, 2, 1.0, 17, eval=ev)
        sums.append(zi.cube_estimates(rq, 0, uids)[2])
    diff = float(np.sum(sums[0] - sums[1]))
    mean_rel = diff / float(np.sum(sums[1]))
    per_sum = float(np.max(np.abs(sums[0] - sums[1]) / np.abs(sums[1])))
    print("FP32 %s: signed mean error %.3g of mean f; largest per-sum error %.3g" % (name, mean_rel, per_sum))
    assert abs(mean_rel) < 1e-6
    assert per_sum < 2e-5


def test_fp32_oscillatory_has_no_mean_error(zi):
    """The oscillatory family (cos of a phase that sweeps many periods over
    the box, so the mean of |f| is 2/pi): signed mean error of FP32 against
    FP64 on the same 5e7 points below 1e-8 of mean |f|."""
    from paper_1902_07916_amd import make_request
    d, D, N, n1 = 8, 4, 4096, 3
    prm = [0.3, 11.0, 17.5, 7.0, 23.0]
    uids = np.arange(d ** D, dtype=np.uint64)
    sums = []
    for ev in ("fp32", "fp64"):
        rq = make_request("genz_osc", prm, [0.0] * D, [1.0] * D, d, N, n1, 2, 1.0, 19, eval=ev)
        sums.append(zi.cube_estimates(rq, 0, uids)[2])
    diff = sums[0] - sums[1]
    n = diff.size * N
    mean_rel = float(np.sum(diff)) / n / (2 / np.pi)
    per_sum = float(np.sqrt(np.mean(diff ** 2))) / N / (2 / np.pi)
    print("FP32 genz_osc: signed mean error %.3g of mean |f|; per-sum rms %.3g" % (mean_rel, per_sum))
    assert abs(mean_rel) < 1e-8
    assert per_sum < 2e-6
