"""Pins of the oracle's method variants (the paper's other readings of
Sec. 2.1): a split into b parts per axis (b^D children; b = d is the paper's
split into k equal parts) and a threshold per parent (over the children of
one split cube) instead of per level."""
import math

import numpy as np
import pytest

import closed_forms as cf


def test_hand_worked_base3_child(orc):
    # D=2, d=2, b=3 on [0,1]^2: root 2 is (K0,K1)=(1,0); child c=5 = digits (1,2)
    p = orc.problem(orc.CONST, 2, 0.0, 1.0, 2, 4, 2, 2, 1.0, 1, params=[1.0], split=3)
    uid = 2 * 9 + 5
    assert list(orc.lattice(2, 2, 1, uid, split=3)) == [4, 2]
    lo, h, v = orc.bounds(p, 1, uid)
    assert h[0] == 0.5 / 3 and lo[0] == pytest.approx(4 / 6, rel=1e-15) and lo[1] == pytest.approx(2 / 6, rel=1e-15)
    uid2 = uid * 9 + 8          # digits (2, 2) -> K = (14, 8) on a 18-cell grid
    assert list(orc.lattice(2, 2, 2, uid2, split=3)) == [14, 8]
    assert list(orc.children(7, 2, split=3)) == [7 * 9 + c for c in range(9)]


@pytest.mark.parametrize("D,d,b", [(2, 2, 3), (3, 3, 3), (2, 3, 4), (4, 2, 2)])
def test_children_tile_parent_bway(orc, D, d, b):
    lower = np.linspace(-1.0, 0.5, D)
    upper = lower + np.linspace(1.0, 2.0, D)
    p = orc.problem(orc.CONST, D, lower, upper, d, 4, 2, 3, 1.0, 1, params=[1.0], split=b)
    rng = np.random.default_rng(D * 7 + b)
    for _ in range(4):
        level = int(rng.integers(0, 3))
        uid = int(rng.integers(0, d**D))
        for _l in range(level):
            uid = uid * b**D + int(rng.integers(0, b**D))
        plo, ph, pv = orc.bounds(p, level, uid)
        kids = orc.children(uid, D, split=b)
        cells = set()
        vol = 0.0
        for c, k in enumerate(kids):
            lo, h, v = orc.bounds(p, level + 1, int(k))
            assert np.allclose(h, ph / b, rtol=1e-15)
            digits = [(c // b ** (D - 1 - i)) % b for i in range(D)]
            assert np.allclose(lo, plo + np.array(digits) * h, rtol=0, atol=4e-16 * (np.abs(upper) + np.abs(lower)))
            cells.add(tuple(digits))
            vol += v
        assert len(cells) == b**D and vol == pytest.approx(pv, rel=1e-14)


@pytest.mark.parametrize("split,scope", [(3, 0), (2, 1), (3, 1)])
def test_variants_match_closed_form(orc, split, scope):
    prm = [2.0, 4.0, 1.0, 0.2, 0.7, 0.9]
    p = orc.problem(orc.GENZ_PPEAK, 3, 0.0, 1.0, 3, 1024, 5, 2, 1.0, 11, params=prm, split=split, scope=scope)
    r = orc.integrate(p)
    assert r.status == 0 and len(r.levels) == 3
    exact = cf.exact(3, prm, [0.0] * 3, [1.0] * 3)
    assert abs(r.integral - exact) <= 5 * r.stderr


def test_per_parent_selection_rule(orc):
    p = orc.problem(orc.GAUSS, 2, -1.0, 1.0, 6, 256, 4, 3, 0.5, 3, params=[0.15, 1.0, 0.1, -0.3], scope=1)
    r = orc.integrate(p)
    assert len(r.levels) >= 3
    L0 = r.levels[0]
    thr0, _, _ = orc.threshold(L0.s, 0.5)
    assert np.array_equal(L0.sel.astype(bool), L0.s > thr0)
    for L in r.levels[1:-1]:
        g = 4  # 2^D siblings per parent
        s = L.s.reshape(-1, g)
        thr = s.mean(axis=1) + 0.5 * s.std(axis=1)
        sel = L.sel.reshape(-1, g).astype(bool)
        away = np.abs(s - thr[:, None]) > 1e-12 * np.abs(thr[:, None])
        assert np.array_equal(sel[away], (s > thr[:, None])[away])
        # Cantelli within every sibling group
        assert np.all(sel.sum(axis=1) <= math.floor(g / (1 + 0.5**2)))
        assert math.isnan(L.thr)


def test_variant_validation(orc):
    base = dict(integrand=orc.GAUSS, dim=2, lower=-1.0, upper=1.0, divisions=4, samples=16, trials=3, max_depth=1,
                sigma_mult=1.0, seed=1, params=[0.2, 1.0, 0.0, 0.0])
    assert orc.validate(orc.problem(**base, split=3, scope=1)) == 0
    for bad in (dict(split=1), dict(split=65), dict(scope=2), dict(split=64, dim=5, params=[0.2, 1.0] + [0.0] * 5)):
        kw = dict(base)
        kw.update(bad)
        assert orc.validate(orc.problem(**kw)) == orc.EINVAL, bad
    # id range (84 bits) with b = 5 in 4-D: 4^4 * 625^8 < 2^84 <= 4^4 * 625^9
    b4 = dict(base, dim=4, params=[0.2, 1.0] + [0.0] * 4)
    assert 4 ** 4 * 625 ** 8 < 2 ** 84 <= 4 ** 4 * 625 ** 9
    assert orc.validate(orc.problem(**dict(b4, max_depth=8), split=5)) == 0
    assert orc.validate(orc.problem(**dict(b4, max_depth=9), split=5)) == orc.EINVAL
