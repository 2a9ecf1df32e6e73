"""Tuning files change speed, not results: every occupancy variant of a
sampling kernel gives bitwise the same integration, and a different cap on
the points per sampling unit (which changes only the order of the FP64
partial sums) agrees to rounding."""
import json
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu


def _run(tmp_path, table, w):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_07916_amd import Integrator
    path = tmp_path / ("tune_%d.json" % abs(hash(json.dumps(table, sort_keys=True))))
    path.write_text(json.dumps(table))
    z = Integrator(arena_bytes=1 << 30, tune_path=str(path))
    try:
        return z.integrate(**w)
    finally:
        z.close()


def _cases():
    from paper_1902_07916_amd import workloads as W
    sin = dict(W.sin6d(eval="fp32", samples=3000, divisions=3, max_depth=2), seed=4)
    gauss = dict(integrand=0, params=[0.1, 1.0] + [0.5] * 5, lower=[0.0] * 5, upper=[1.0] * 5, divisions=3,
                 samples=2500, trials=5, max_depth=2, sigma_mult=0.5, seed=2, eval="fp32")
    osc64 = dict(integrand=2, params=[0.2, 3.0, 1.0, 2.0, 0.5], lower=[0.0] * 4, upper=[1.0] * 4, divisions=4,
                 samples=2000, trials=4, max_depth=2, sigma_mult=0.5, seed=3, eval="fp64")
    return {"sin6d_fp32": (sin, "1:6:1"), "gauss5d_fp32": (gauss, "0:5:1"), "osc4d_fp64": (osc64, "2:4:0")}


@pytest.mark.parametrize("case", ["sin6d_fp32", "gauss5d_fp32", "osc4d_fp64"])
def test_occupancy_variants_bitwise(tmp_path, case):
    w, key = _cases()[case]
    print("tuning: %s across occupancy variants" % case, flush=True)
    ref = None
    for waves in (1, 5, 7, 8):
        r = _run(tmp_path, {key + ":w": waves}, w)
        assert r.status == 0
        got = (r.integral, r.std, tuple(r.cubes_per_level), tuple(r.selected_per_level))
        if ref is None:
            ref = got
        assert got == ref, (waves, got, ref)


def test_unit_size_changes_only_rounding(tmp_path):
    w, key = _cases()["sin6d_fp32"]
    print("tuning: sin6d across unit sizes", flush=True)
    base = _run(tmp_path, {key: 32}, w)
    for groups in (2, 4, 8):
        r = _run(tmp_path, {key: groups}, w)
        assert r.status == 0
        assert tuple(r.cubes_per_level) == tuple(base.cubes_per_level)
        assert abs(r.integral - base.integral) <= 1e-12 * max(abs(base.integral), base.std)
        assert abs(r.std - base.std) <= 1e-12 * base.std
