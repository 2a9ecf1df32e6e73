"""Pins of the oracle's cube ids beyond 64 bits (up to 84).  Counter word 1
of a cube's Philox stream carries the trial in bits 0..7, the level in bits
8..11 and id bits 64..83 in bits 12..31, so ids below 2^64 keep their
streams; the lattice decode and the children follow the same arithmetic on
the wider ids.  Used by deep bisection trees (root bits + D per level > 64)
and by the paper's 12-D Gaussian of Table 4 at its depth 4 (3^12 roots,
three 3^12-way splits: ids below 3^48 ~ 2^76.1)."""
import numpy as np
import pytest


def test_counter_layout_of_wide_ids(orc):
    seed = 0x0123456789ABCDEF
    for uid in (5, (1 << 64) + 7, (3 ** 48 - 1) // 2, (1 << 84) - 1):
        lo, hi = uid & ((1 << 64) - 1), uid >> 64
        for level, trial, D, s, i in ((0, 0, 3, 0, 0), (3, 4, 12, 17, 5), (15, 254, 7, 1001, 6)):
            n = s * D + i
            ctr = (n >> 2, trial | (level << 8) | (hi << 12), lo & 0xFFFFFFFF, lo >> 32)
            want = orc.philox(ctr, (seed & 0xFFFFFFFF, seed >> 32))[n & 3]
            assert orc.word(seed, uid, level, trial, D, s, i) == want
    with pytest.raises(ValueError):
        orc.word(seed, 1 << 84, 0, 0, 1, 0, 0)


def test_centre_cube_of_the_12d_depth4_tree(orc):
    # [-1,1]^12, 3 parts per axis at the root and per split: the centre cube
    # at level 3 has base-3^12 digits all (3^12 - 1) / 2, i.e. every axis
    # digit 1: K = 1*27 + 1*9 + 1*3 + 1 = 40 on 81 cells per axis
    D, d, b = 12, 3, 3
    k = 3 ** D
    centre = (k - 1) // 2
    uid = ((centre * k + centre) * k + centre) * k + centre
    assert uid == (3 ** 48 - 1) // 2 and uid >> 64 > 0
    assert list(orc.lattice(D, d, 3, uid, split=b)) == [40] * D
    p = orc.problem(orc.GAUSS, D, -1.0, 1.0, d, 4, 2, 3, 4.0, 1, params=[0.01, 1.0] + [0.0] * D, split=b)
    lo, h, v = orc.bounds(p, 3, uid)
    assert np.allclose(h, 2.0 / 81, rtol=1e-15) and np.allclose(lo, -1.0 / 81, rtol=0, atol=1e-15)
    # its children: uid * 3^12 + c, with the id bits above 64 carried
    clo, chi = orc.children_w(uid, D, b)
    for c in (0, 1, 265720, k - 1):
        want = uid * k + c
        assert int(clo[c]) == want & ((1 << 64) - 1) and int(chi[c]) == want >> 64


def test_deep_bisection_ids(orc):
    # D = 6, d = 4: 12 root bits + 6 per split, past 64 bits at level 9.  Root
    # 4095 (every axis cell 3) and path bits all one: K = 3 * 2^9 + 511 = 2047
    D, d, level = 6, 4, 9
    uid = (4095 << (D * level)) | ((1 << (D * level)) - 1)
    assert uid >> 64 > 0
    assert list(orc.lattice(D, d, level, uid)) == [2047] * D
    p = orc.problem(orc.CONST, D, -1.0, 1.0, d, 4, 2, 11, 1.0, 1, params=[1.0])
    lo, h, v = orc.bounds(p, level, uid)
    assert np.all(h == 2.0 / 2048) and np.all(lo == -1.0 + 2047 * (2.0 / 2048))
    clo, chi = orc.children_w(uid, D, 2)
    for c in (0, 5, 63):
        want = (uid << D) | c
        assert int(clo[c]) == want & ((1 << 64) - 1) and int(chi[c]) == want >> 64
    # a sample point of the wide cube lies inside it
    x = orc.sample_x(p, level, uid, 1, 3)
    assert np.all(x > lo) and np.all(x < lo + h)


def test_tree_through_wide_ids(orc):
    # a narrow product peak followed to level 11: levels 10 and 11 hold ids
    # past 2^64; each level's list is the children of the previous level's
    # selected cubes (as Python integers), and the estimate of a wide-id cube
    # agrees with the closed form of that cube's integral
    import closed_forms as cf
    prm = [1e3] * 6 + [0.3141, 0.2718, 0.5772, 0.6931, 0.4142, 0.7320]
    p = orc.problem(orc.GENZ_PPEAK, 6, 0.0, 1.0, 4, 256, 4, 11, 3.0, 3, params=prm)
    r = orc.integrate(p)
    assert r.status == 0 and len(r.levels) == 12
    assert r.levels[10].uid_hi.max() > 0 and r.levels[11].uid_hi.max() > 0
    for L, Ln in zip(r.levels[:-1], r.levels[1:]):
        ids = [int(u) | (int(h) << 64) for u, h in zip(L.uid, L.uid_hi)]
        nxt = [int(u) | (int(h) << 64) for u, h in zip(Ln.uid, Ln.uid_hi)]
        want = [(i << 6) | c for i, s in zip(ids, L.sel) if s for c in range(64)]
        assert nxt == want
    L = r.levels[11]
    for c in (0, int(np.argmax(L.uid_hi))):
        uid = int(L.uid[c]) | (int(L.uid_hi[c]) << 64)
        lo, h, v = orc.bounds(p, 11, uid)
        exact = cf.exact(3, prm, lo, lo + h)
        assert abs(L.m[c] - exact) <= 6 * L.s[c] / np.sqrt(3) + 1e-12 * abs(exact), (c, L.m[c], exact, L.s[c])
