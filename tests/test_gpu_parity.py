"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs, step by step (RNG words, sample points, per-(cube, trial)
sums, per-cube mean/std, threshold, selection, children) and end to end.

Tolerances: FP64 evaluation -- integral/std within 1e-6 relative (expected
~1e-12; differences come only from summation order and libm ulps); FP32
evaluation -- within 1e-4 relative of the FP64 oracle.  Selections and child
lists are compared bit-exactly outside a margin band around the threshold
(|s - thr| / thr <= eps, eps = 1e-9 for FP64, 1e-4 for FP32); decisions
inside the band are adopted by the oracle's replay mode."""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from common import compare_tree, oracle_problem, rel, request  # noqa: E402

pytestmark = pytest.mark.gpu

EPS64 = 1e-9
EPS32 = 1e-4


@pytest.fixture(scope="module")
def zi():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_07916_amd import Integrator
    z = Integrator(arena_bytes=8 << 30)
    yield z
    z.close()


def _compare_tree(orc, w, r, eps, tol):
    return compare_tree(orc, w, r, eps, tol)


def test_philox_words_bitwise(zi, orc):
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2**32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    key = (0x9ABCDEF0, 0x12345678)
    out = zi.debug_philox(key, ctr)
    for i in range(0, 4096, 97):
        assert tuple(out[i]) == orc.philox(ctr[i], key)


def test_sample_points_bitwise(zi, orc):
    from paper_1902_07916_amd import workloads as W
    for w in (W.gauss4d(), W.sin6d(), W.narrow_gauss9d()):
        req = request(w)
        p = oracle_problem(orc, w)
        D = len(w["lower"])
        for level, uid in ((0, 0), (0, 17), (1, (5 << D) | 3), (2, (((7 << D) | 1) << D) | ((1 << D) - 1))):
            x = zi.debug_points(req, level, uid, 2, 123, 9)
            for k in range(9):
                assert np.array_equal(x[k], orc.sample_x(p, level, uid, 2, 123 + k)), (w["integrand"], level, k)


@pytest.mark.parametrize("eval_", ["fp64", "fp32"])
def test_cube_sums_gauss4d(zi, orc, eval_):
    from paper_1902_07916_amd import workloads as W
    w = W.gauss4d(eval=eval_)
    req = request(w)
    p = oracle_problem(orc, w)
    uids = np.array([0, 5, 85, 170, 255], dtype=np.uint64)
    m, s, S1, S2 = zi.cube_estimates(req, 0, uids)
    tol = 1e-12 if eval_ == "fp64" else 1e-5
    for i, u in enumerate(uids):
        st, I, mo, so, _ = orc.cube(p, 0, int(u))
        for t in range(w["trials"]):
            _, It, S1o, S2o, _ = orc.cube_trial(p, 0, int(u), t)
            assert rel(S1[i, t], S1o) < tol, (i, t)
            assert rel(S2[i, t], S2o) < tol * 10
        assert rel(m[i], mo) < tol
        assert abs(s[i] - so) < tol * 100 * abs(mo) + 1e-300


def test_gauss4d_full_tree_fp64(zi, orc):
    from paper_1902_07916_amd import workloads as W
    w = W.gauss4d(eval="fp64")
    r = zi.integrate(**w, trace=True)
    o = _compare_tree(orc, w, r, EPS64, 1e-6)
    assert rel(r.integral, o.integral) < 1e-11
    assert o.levels[0].n_in_band == 0
    assert r.n_samples == o.n_samples and r.n_cubes == o.n_cubes


def test_gauss4d_full_tree_fp32(zi, orc):
    from paper_1902_07916_amd import workloads as W
    w = W.gauss4d(eval="fp32")
    r = zi.integrate(**w, trace=True)
    _compare_tree(orc, w, r, EPS32, 1e-4)


SMALL = [
    ("gauss", dict(integrand=0, params=[0.3, 2.0, 0.1, -0.2, 0.3], lower=[-1.0, -0.5, 0.0], upper=[1.0, 1.5, 0.5])),
    ("sin_sum", dict(integrand=1, params=[], lower=[0.0, 1.0, -2.0], upper=[4.0, 3.5, 3.0])),
    ("genz_osc", dict(integrand=2, params=[0.3, 1.0, 2.5, 0.7, 4.0], lower=[0.0] * 4, upper=[1.0] * 4)),
    ("genz_ppeak", dict(integrand=3, params=[2.0, 4.0, 1.0, 0.2, 0.7, 0.9], lower=[0.0] * 3, upper=[1.0] * 3)),
    ("genz_cpeak", dict(integrand=4, params=[0.9, 2.0, 3.5], lower=[0.0] * 3, upper=[1.0] * 3)),
    ("genz_gauss", dict(integrand=5, params=[1.0, 3.0, 0.5, 2.0, 0.2, 0.8, 0.5, 0.1], lower=[0.0] * 4,
                        upper=[1.0] * 4)),
    ("const", dict(integrand=6, params=[1.25], lower=[0.0] * 2, upper=[2.0] * 2)),
    ("monomial", dict(integrand=7, params=[1.0, 2.0, 3.0], lower=[0.0, -1.0, 0.5], upper=[1.0, 2.0, 1.5])),
]


@pytest.mark.parametrize("eval_", ["fp64", "fp32"])
@pytest.mark.parametrize("name,base", SMALL, ids=[s[0] for s in SMALL])
def test_every_integrand_small_tree(zi, orc, name, base, eval_):
    # 3 divisions, N = 3001 (several chunks of 1024 groups? no: a ragged
    # 4-point group and a partial chunk), 2 refinements
    w = dict(base, divisions=3, samples=3001, trials=4, max_depth=2, sigma_mult=1.0, seed=77, eval=eval_)
    r = zi.integrate(**w, trace=True)
    _compare_tree(orc, w, r, EPS64 if eval_ == "fp64" else EPS32, 1e-6 if eval_ == "fp64" else 1e-4)


def test_constant_integrand_exact(zi):
    r = zi.integrate("const", [1.5], [-1.0] * 4, [1.0] * 4, 4, 4096, 5, 3, 1.0, 1, eval="fp64")
    assert r.integral == 24.0 and r.std == 0.0 and r.levels_run == 1
    assert r.selected_per_level == [0]


def test_nonfinite_integrand(zi):
    from paper_1902_07916_amd import ZmcError
    with pytest.raises(ZmcError) as e:
        zi.integrate("const", [float("nan")], [0.0] * 2, [1.0] * 2, 2, 8, 3, 1, 1.0, 1)
    assert e.value.code == -3


@pytest.mark.parametrize("case", [
    dict(integrand=1, params=[], lower=[0.0], upper=[3.0], divisions=5, samples=1, trials=2, max_depth=3),
    dict(integrand=1, params=[], lower=[0.0], upper=[3.0], divisions=1, samples=7, trials=255, max_depth=0),
    dict(integrand=0, params=[0.5, 1.0] + [0.1] * 16, lower=[-1.0] * 16, upper=[1.0] * 16, divisions=1,
         samples=5, trials=3, max_depth=1),
    dict(integrand=3, params=[3.0] * 12 + [0.4] * 12, lower=[0.0] * 12, upper=[1.0] * 12, divisions=2,
         samples=12, trials=3, max_depth=1),
])
def test_edge_shapes(zi, orc, case):
    w = dict(case, sigma_mult=1.0, seed=3, eval="fp64")
    r = zi.integrate(**w, trace=True, trace_capacity=1 << 22)
    _compare_tree(orc, w, r, EPS64, 1e-6)


def test_truncation_and_rtol(zi, orc):
    w = dict(integrand=1, params=[], lower=[0.0] * 2, upper=[6.0] * 2, divisions=8, samples=256, trials=4,
             max_depth=3, sigma_mult=0.0, seed=5, eval="fp64", max_cubes_per_level=64)
    r = zi.integrate(**w, trace=True)
    o = orc.integrate(oracle_problem(orc, w))
    assert r.flags == o.flags == 1
    assert rel(r.integral, o.integral) < 1e-9
    w = dict(integrand=0, params=[0.3, 1.0, 0.0, 0.0], lower=[-1.0] * 2, upper=[1.0] * 2, divisions=4,
             samples=1024, trials=3, max_depth=4, sigma_mult=1.0, seed=5, eval="fp64", rtol=1e-2)
    r = zi.integrate(**w)
    o = orc.integrate(oracle_problem(orc, w))
    assert r.flags == o.flags == 2 and r.levels_run == len(o.levels)
    assert rel(r.integral, o.integral) < 1e-9


def test_deterministic_run_to_run(zi):
    from paper_1902_07916_amd import workloads as W
    w = W.sin6d(eval="fp32", samples=2048, divisions=4, max_depth=2)
    a = zi.integrate(**w)
    b = zi.integrate(**w)
    assert a.integral == b.integral and a.std == b.std and a.cubes_per_level == b.cubes_per_level


@pytest.mark.parametrize("eval_", ["fp64", "fp32"])
def test_tree_through_wide_ids(zi, orc, eval_):
    """Cube ids past 64 bits (bits 64..83 in a second array and in counter
    word 1): a narrow 6-D product peak followed by bisection to level 11
    (12 root bits + 6 per split), whose levels 10 and 11 hold such ids;
    the whole tree against the oracle, id lists bit-exact."""
    prm = [1e3] * 6 + [0.3141, 0.2718, 0.5772, 0.6931, 0.4142, 0.7320]
    w = dict(integrand=3, params=prm, lower=[0.0] * 6, upper=[1.0] * 6, divisions=4, samples=256, trials=4,
             max_depth=11, sigma_mult=3.0, seed=3, eval=eval_)
    r = zi.integrate(**w, trace=True)
    assert r.levels_run == 12
    assert r.trace[10]["uid_hi"].max() > 0 and r.trace[11]["uid_hi"].max() > 0
    _compare_tree(orc, w, r, EPS64 if eval_ == "fp64" else EPS32, 1e-6 if eval_ == "fp64" else 1e-4)


def test_bway_tree_through_wide_ids(zi, orc):
    """Ids past 64 bits under a b-way split (b = 64, 4096 children per
    cube): a very narrow 2-D product peak on 8 x 8 roots, split to level 5
    (6 root bits + 12 per split), whose last level holds ids above 2^64 (the
    decode divides a 128-bit id by 4096 per level).  FP64 evaluation: in
    FP32 the peak's values at the root level lie below FP32's range.  The
    whole tree against the oracle, id lists bit-exact."""
    w = dict(integrand=3, params=[1e11, 1e11, 0.3141592, 0.2718281], lower=[0.0, 0.0], upper=[1.0, 1.0],
             divisions=8, samples=64, trials=2, max_depth=5, sigma_mult=3.0, seed=5, split=64,
             max_cubes_per_level=1 << 14, eval="fp64")
    r = zi.integrate(**w, trace=True)
    assert r.levels_run == 6 and not r.flags & 1
    assert r.trace[5]["uid_hi"].max() > 0
    _compare_tree(orc, w, r, EPS64, 1e-6)
