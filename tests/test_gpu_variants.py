"""GPU parity of the tree-search variants against the oracle: k-way splits
(every axis cut into b equal parts, b^D children; Sec. 2.1 splits a cube into k
equal parts) and per-parent thresholds (a new threshold from each
split cube's own children), alone and combined, FP64 and FP32 evaluation.

Same bar as the bisection parity tests: lists bit-exact, per-cube m and s
within 1e-6 (FP64) / 1e-4 (FP32) relative, selections exact outside the
margin band around each cube's own threshold, decisions inside it replayed
by the oracle."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from common import compare_tree  # noqa: E402

pytestmark = pytest.mark.gpu

EPS64 = 1e-9
EPS32 = 1e-4


@pytest.fixture(scope="module")
def zi():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_07916_amd import Integrator
    z = Integrator(arena_bytes=4 << 30)
    yield z
    z.close()


def _compare(orc, w, r, eps, tol):
    return compare_tree(orc, w, r, eps, tol)


def _w(integrand, params, D, lo, hi, d, N, depth, sm, split, scope, eval_, seed=3):
    return dict(integrand=integrand, params=params, lower=[lo] * D, upper=[hi] * D, divisions=d, samples=N,
                trials=5, max_depth=depth, sigma_mult=sm, seed=seed, eval=eval_, split=split, scope=scope)


CASES = {
    # 3-way split of a 3-D Gaussian: 27 children per split cube
    "split3_gauss3d": lambda ev: _w(0, [0.15, 1.0, 0.1, 0.0, -0.1], 3, -1.0, 1.0, 3, 2000, 2, 0.5, 3, 0, ev),
    # per-parent thresholds with bisection, 4-D Gaussian, three refinements
    "scope1_gauss4d": lambda ev: _w(0, [0.2, 1.0, 0.0, 0.0, 0.0, 0.0], 4, -1.0, 1.0, 3, 1500, 3, 0.5, 0, 1, ev),
    # both at once, 2-D oscillatory with 5-way splits (25 children)
    "split5_scope1_osc2d": lambda ev: _w(2, [0.25, 6.0, 9.0], 2, 0.0, 1.0, 4, 1500, 3, 0.0, 5, 1, ev),
    # ragged: split 7 on a 2-D corner peak, 49 children (not a tile multiple)
    "split7_cpeak2d": lambda ev: _w(4, [3.0, 2.0], 2, 0.0, 1.0, 2, 777, 3, 0.0, 7, 0, ev),
    # degenerate per-parent case: one parent per level (levels of 16, 4, 4, 4
    # cubes), so each level's only sibling group is the whole level
    "scope1_single_parent": lambda ev: _w(0, [0.03, 1.0, 0.3, 0.3], 2, 0.0, 1.0, 4, 2000, 3, 1.0, 0, 1, ev),
}


@pytest.mark.parametrize("eval_", ["fp64", "fp32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_variant_tree(zi, orc, case, eval_):
    w = CASES[case](eval_)
    r = zi.integrate(**w, trace=True)
    assert r.levels_run == w["max_depth"] + 1, "tree stopped early; the case does not exercise every level"
    if eval_ == "fp64":
        _compare(orc, w, r, EPS64, 1e-6)
    else:
        _compare(orc, w, r, EPS32, 1e-4)


def test_split2_explicit_equals_default(zi):
    """split = 2 is bisection: bitwise the same run as split = 0."""
    w = CASES["scope1_gauss4d"]("fp64")
    a = zi.integrate(**dict(w, split=0))
    b = zi.integrate(**dict(w, split=2))
    assert a.integral == b.integral and a.std == b.std
    assert list(a.cubes_per_level) == list(b.cubes_per_level)


def test_variant_batch_matches_alone(zi):
    """Variants mixed with plain requests in one batch give bitwise the same
    results as each request alone."""
    from paper_1902_07916_amd import request_from_dict
    ws = [CASES[c]("fp64") for c in sorted(CASES)] + [
        _w(0, [0.2, 1.0, 0.0, 0.0, 0.0, 0.0], 4, -1.0, 1.0, 3, 1500, 3, 0.5, 0, 0, "fp64")]
    reqs = [request_from_dict(w) for w in ws]
    batch = zi.integrate_batch(reqs)
    for w, rb in zip(ws, batch):
        ra = zi.integrate(**w)
        assert rb.integral == ra.integral and rb.std == ra.std, w
        assert list(rb.cubes_per_level) == list(ra.cubes_per_level)


def test_variant_argument_errors(zi):
    from paper_1902_07916_amd import ZmcError
    w = CASES["split3_gauss3d"]("fp64")
    for bad in (dict(split=1), dict(split=65), dict(scope=2), dict(split=64, lower=[0.0] * 5, upper=[1.0] * 5,
                                                                       params=[0.15, 1.0] + [0.0] * 5)):
        with pytest.raises(ZmcError):
            zi.integrate(**dict(w, **bad))
