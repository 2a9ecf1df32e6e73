"""Pins of the oracle's sub-domain geometry: hand-worked lattice cases, children
that tile their parent, leaves that tile the domain, samples inside their cube."""
import itertools

import numpy as np
import pytest


def test_hand_worked_root_order(orc):
    # D=2, d=4 on [-1,1]^2: root r = 4*K0 + K1 (axis 0 most significant), edge 0.5
    p = orc.problem(orc.CONST, 2, -1.0, 1.0, 4, 4, 2, 1, 1.0, 1, params=[1.0])
    lo, h, v = orc.bounds(p, 0, 1)
    assert list(lo) == [-1.0, -0.5] and list(h) == [0.5, 0.5] and v == 0.25
    lo, h, v = orc.bounds(p, 0, 4)
    assert list(lo) == [-0.5, -1.0]
    lo, h, v = orc.bounds(p, 0, 15)
    assert list(lo) == [0.5, 0.5]


def test_hand_worked_child(orc):
    # D=2, d=2 on [0,1]^2, level 1: root 2 is (K0,K1)=(1,0); child c=1 has bits (0,1)
    p = orc.problem(orc.CONST, 2, 0.0, 1.0, 2, 4, 2, 2, 1.0, 1, params=[1.0])
    uid = (2 << 2) | 1
    assert list(orc.lattice(2, 2, 1, uid)) == [2, 1]
    lo, h, v = orc.bounds(p, 1, uid)
    assert list(lo) == [0.5, 0.25] and list(h) == [0.25, 0.25] and v == 0.0625
    # level 2: child 3 (bits 1,1) of that cube -> K = (5, 3), edge 1/8
    uid2 = (uid << 2) | 3
    assert list(orc.lattice(2, 2, 2, uid2)) == [5, 3]
    lo, h, v = orc.bounds(p, 2, uid2)
    assert list(lo) == [0.625, 0.375] and list(h) == [0.125, 0.125]


@pytest.mark.parametrize("D,d", [(1, 3), (2, 2), (3, 5), (4, 2), (6, 3)])
def test_children_tile_parent(orc, D, d):
    lower = np.linspace(-1.5, 0.25, D)
    upper = lower + np.linspace(1.0, 3.0, D)
    p = orc.problem(orc.CONST, D, lower, upper, d, 4, 2, 3, 1.0, 1, params=[1.0])
    rng = np.random.default_rng(D * 100 + d)
    for _ in range(5):
        level = int(rng.integers(0, 3))
        uid = int(rng.integers(0, d**D))
        for _l in range(level):
            uid = (uid << D) | int(rng.integers(0, 2**D))
        plo, ph, pv = orc.bounds(p, level, uid)
        kids = orc.children(uid, D)
        assert len(kids) == 2**D and np.all(np.diff(kids.astype(np.float64)) > 0)
        vols = 0.0
        corners = set()
        for c, k in enumerate(kids):
            lo, h, v = orc.bounds(p, level + 1, int(k))
            assert np.all(h == ph / 2)
            # child sits in the half given by bit (D-1-i) of c along axis i
            for i in range(D):
                bit = (c >> (D - 1 - i)) & 1
                want = plo[i] + h[i] if bit else plo[i]
                assert lo[i] == pytest.approx(want, rel=0, abs=4e-16 * (abs(upper[i]) + abs(lower[i])))
            corners.add(tuple(lo))
            vols += v
        assert len(corners) == 2**D
        assert vols == pytest.approx(pv, rel=1e-15)


def test_leaves_tile_dyadic_domain_exactly(orc):
    # Constant integrand with a random-looking tree forced by replay: accepted
    # leaf volumes sum to the domain volume exactly (dyadic edges).
    p = orc.problem(orc.GAUSS, 3, -1.0, 1.0, 2, 64, 3, 3, 0.5, 9, params=[0.3, 1.0, 0.1, -0.2, 0.3])
    r = orc.integrate(p)
    assert r.status == 0 and len(r.levels) >= 2
    total = 0.0
    for l, L in enumerate(r.levels):
        for uid, sel in zip(L.uid, L.sel):
            if not sel:
                total += orc.bounds(p, l, int(uid))[2]
    assert total == 8.0


def test_samples_inside_cube(orc):
    p = orc.problem(orc.SIN_SUM, 4, [0, -3, 2, 5], [1, 3, 2.5, 9], 3, 50, 3, 2, 1.0, 77)
    for level, uid in [(0, 0), (0, 80), (1, (17 << 4) | 9), (2, (((40 << 4) | 15) << 4) | 0)]:
        lo, h, _ = orc.bounds(p, level, uid)
        for t in range(3):
            for s in range(50):
                x = orc.sample_x(p, level, uid, t, s)
                assert np.all(x > lo) and np.all(x < lo + h)


def test_level_lists_ascending(orc):
    p = orc.problem(orc.GAUSS, 2, -1.0, 1.0, 4, 256, 4, 3, 0.5, 3, params=[0.2, 1.0, 0.0, 0.0])
    r = orc.integrate(p)
    for L in r.levels:
        assert np.all(np.diff(L.uid.astype(object)) > 0) if L.n > 1 else True
