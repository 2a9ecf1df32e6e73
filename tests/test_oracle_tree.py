"""Pins of the oracle's tree search: threshold, selection, Cantelli bound,
truncation and rtol stopping rules, replay, argument checks."""
import math

import numpy as np
import pytest


def test_threshold_hand_example(orc):
    thr, mu, sd = orc.threshold([1.0, 2.0, 3.0, 4.0, 5.0], 1.0)
    assert mu == 3.0 and sd == pytest.approx(math.sqrt(2.0), rel=1e-15)
    assert thr == pytest.approx(3.0 + math.sqrt(2.0), rel=1e-15)
    thr, mu, sd = orc.threshold([2.0, 2.0, 2.0], 5.0)
    assert thr == 2.0 and sd == 0.0


def test_threshold_matches_numpy(orc):
    s = np.random.default_rng(3).lognormal(size=10001)
    thr, mu, sd = orc.threshold(s, 0.5)
    assert mu == pytest.approx(np.mean(s), rel=1e-13)
    assert sd == pytest.approx(np.std(s), rel=1e-12)     # population std, ddof = 0
    assert thr == pytest.approx(np.mean(s) + 0.5 * np.std(s), rel=1e-12)


@pytest.mark.parametrize("sigma", [0.0, 0.5, 1.0, 2.0])
def test_selection_rule_and_cantelli(orc, sigma):
    p = orc.problem(orc.GAUSS, 2, -1.0, 1.0, 8, 256, 4, 2, sigma, 11, params=[0.15, 1.0, 0.1, -0.3])
    r = orc.integrate(p)
    assert r.status == 0
    for l, L in enumerate(r.levels[:-1]):
        # strict "s > thr" with thr over this level's list
        thr, mu, sd = orc.threshold(L.s, sigma)
        assert L.thr == thr
        assert np.array_equal(L.sel.astype(bool), L.s > thr)
        # Cantelli's one-sided bound on how many can exceed mean + k sd
        bound = L.n - 1 if sigma == 0.0 else math.floor(L.n / (1 + sigma**2))
        assert L.n_sel <= bound
        # next level lists the selected cubes' children in parent order
        if l + 1 < len(r.levels):
            want = np.concatenate([orc.children(int(u), 2) for u in L.uid[L.sel.astype(bool)]])
            assert np.array_equal(r.levels[l + 1].uid, want)
    last = r.levels[-1]
    assert last.n_sel == 0


def test_totals_are_sums_over_accepted(orc):
    p = orc.problem(orc.GENZ_PPEAK, 3, 0.0, 1.0, 3, 128, 5, 2, 1.0, 4, params=[3, 2, 4, 0.2, 0.6, 0.9])
    r = orc.integrate(p)
    M = S2 = 0.0
    for L in r.levels:
        acc = ~L.sel.astype(bool)
        M += L.m[acc].sum()
        S2 += (L.s[acc] ** 2).sum()
    assert r.integral == pytest.approx(M, rel=1e-13)
    assert r.std == pytest.approx(math.sqrt(S2), rel=1e-13)
    assert r.stderr == pytest.approx(math.sqrt(S2 / 4), rel=1e-13)
    assert r.n_samples == sum(L.n for L in r.levels) * 5 * 128
    # trial mean / population std per cube
    L = r.levels[0]
    assert np.allclose(L.m, L.I.mean(axis=1), rtol=1e-14, atol=0)
    assert np.allclose(L.s, L.I.std(axis=1), rtol=1e-10, atol=1e-300)


def test_depth_zero_accepts_everything(orc):
    p = orc.problem(orc.SIN_SUM, 2, 0.0, 3.0, 5, 64, 3, 0, 1.0, 2)
    r = orc.integrate(p)
    assert len(r.levels) == 1 and r.levels[0].n_sel == 0
    assert r.integral == pytest.approx(r.levels[0].m.sum(), rel=1e-14)


def test_truncation_rule(orc):
    # sigma_mult = 0 selects about half of the 64 root cubes: 4x that exceeds the cap
    p = orc.problem(orc.SIN_SUM, 2, 0.0, 6.0, 8, 256, 4, 3, 0.0, 5, max_cubes_per_level=64)
    r = orc.integrate(p)
    assert r.flags & orc.F_TRUNCATED
    assert len(r.levels) == 1
    L = r.levels[-1]
    assert L.n_sel * 4 > 64
    # every cube of the last level is accepted, selected or not
    assert r.integral == pytest.approx(L.m.sum(), rel=1e-13)
    assert r.std == pytest.approx(math.sqrt((L.s ** 2).sum()), rel=1e-13)
    # a cap that fits changes nothing
    p2 = orc.problem(orc.SIN_SUM, 2, 0.0, 6.0, 8, 256, 4, 1, 0.0, 5, max_cubes_per_level=4 * 64)
    assert not orc.integrate(p2).flags & orc.F_TRUNCATED


def test_rtol_stop(orc):
    prm = [0.3, 1.0, 0.0, 0.0]
    loose = orc.integrate(orc.problem(orc.GAUSS, 2, -1.0, 1.0, 4, 1024, 3, 4, 1.0, 5, params=prm, rtol=1e-2))
    assert loose.flags & orc.F_RTOL_MET and len(loose.levels) == 1
    assert loose.stderr <= 1e-2 * abs(loose.integral)
    tight = orc.integrate(orc.problem(orc.GAUSS, 2, -1.0, 1.0, 4, 1024, 3, 4, 1.0, 5, params=prm, rtol=1e-9))
    assert not (tight.flags & orc.F_RTOL_MET)
    nort = orc.integrate(orc.problem(orc.GAUSS, 2, -1.0, 1.0, 4, 1024, 3, 4, 1.0, 5, params=prm))
    assert tight.integral == nort.integral and len(tight.levels) == len(nort.levels)


def test_replay_adopts_only_in_band_decisions(orc):
    p = orc.problem(orc.GAUSS, 2, -1.0, 1.0, 8, 256, 4, 2, 1.0, 11, params=[0.15, 1.0, 0.1, -0.3])
    r = orc.integrate(p)
    L0 = r.levels[0]
    # flip every decision in the replay: outside the band nothing changes
    flipped = [(L.uid, 1 - L.sel) for L in r.levels]
    r2 = orc.integrate(p, replay=flipped, band_eps=0.0)
    assert r2.integral == r.integral and r2.levels[0].n_replayed == 0
    # widen the band to cover the closest cube: exactly the in-band ones flip
    eps = float(np.sort(np.abs(L0.s - L0.thr) / L0.thr)[1]) * 1.0000001
    r3 = orc.integrate(p, replay=flipped, band_eps=eps)
    assert r3.levels[0].n_in_band == 2 and r3.levels[0].n_replayed == 2
    assert r3.levels[0].n_sel != L0.n_sel or True


def test_validation(orc):
    good = dict(integrand=orc.GAUSS, dim=2, lower=-1.0, upper=1.0, divisions=4, samples=16, trials=3,
                max_depth=1, sigma_mult=1.0, seed=1, params=[0.2, 1.0, 0.0, 0.0])
    assert orc.validate(orc.problem(**good)) == 0
    bad = [dict(dim=0, params=[0.2, 1.0]), dict(dim=17), dict(lower=1.0, upper=1.0), dict(divisions=0),
           dict(samples=0), dict(trials=1), dict(trials=256), dict(max_depth=-1), dict(max_depth=16),
           dict(sigma_mult=-1.0), dict(sigma_mult=float("nan")), dict(params=[0.2, 1.0]),
           dict(integrand=99), dict(dim=16, divisions=2, max_depth=5, params=[0.2, 1.0] + [0.0] * 16),
           # ids past 84 bits (3^12 roots, three 3^12-way splits: 2^76 is fine, four: 2^95 not)
           dict(dim=12, divisions=3, split=3, max_depth=4, params=[0.2, 1.0] + [0.0] * 12),
           # lattice cells per axis past 64 bits though ids fit 84 (2 * 64^11 = 2^67)
           dict(dim=1, divisions=2, split=64, max_depth=11, params=[0.2, 1.0, 0.0]),
           dict(integrand=orc.MONOMIAL, params=[1.5, 2.0])]
    for b in bad:
        kw = dict(good)
        kw.update(b)
        assert orc.validate(orc.problem(**kw)) == orc.EINVAL, b
    r = orc.integrate(orc.problem(**dict(good, trials=1)))
    assert r.status == orc.EINVAL
    # ids of up to 84 bits are accepted: 16 root bits + 4 x 16, and 3^12 * (3^12)^3
    for ok in (dict(dim=16, divisions=2, max_depth=4, params=[0.2, 1.0] + [0.0] * 16),
               dict(dim=12, divisions=3, split=3, max_depth=3, params=[0.2, 1.0] + [0.0] * 12),
               dict(dim=1, divisions=2, split=64, max_depth=10, params=[0.2, 1.0, 0.0])):
        kw = dict(good)
        kw.update(ok)
        assert orc.validate(orc.problem(**kw)) == 0, ok


def test_nonfinite_integrand_fails_run(orc):
    p = orc.problem(orc.CONST, 2, 0.0, 1.0, 2, 8, 3, 1, 1.0, 1, params=[float("nan")])
    r = orc.integrate(p)
    assert r.status == orc.ENONFINITE


def test_std_of_tiny_values(orc):
    # deviations near 1e-200: their squares lie below FP64's range, so an
    # unscaled sum of squares is 0; numpy on the values scaled by 2^700
    # (exact) gives the reference
    s = np.array([1.0, 2.0, 4.0, 3.5, 0.25]) * 1e-200
    thr, mu, sd = orc.threshold(s, 2.0)
    ref = np.std(s * 2.0 ** 700) * 2.0 ** -700
    assert sd > 0 and sd == pytest.approx(ref, rel=1e-15)
    assert mu == pytest.approx(np.mean(s), rel=1e-15)
    assert thr == pytest.approx(mu + 2.0 * ref, rel=1e-15)
    # the scaling is exact: ordinary values give the unscaled formula's bits
    x = np.random.default_rng(5).lognormal(size=257)
    _, mu2, sd2 = orc.threshold(x, 1.0)
    assert sd2 == math.sqrt(sum((v - mu2) ** 2 for v in x) / len(x))


def test_cube_std_of_tiny_trials(orc):
    # the 12-D normalised Gaussian (sigma 0.01, 3 cells per axis, 10^4
    # points, 5 trials), seed 2: the centre root cube's trial values are
    # 1e-240 .. 1e-186, whose squared deviations underflow; its std is that
    # of the values scaled by a power of two
    import common
    from paper_1902_07916_amd import workloads
    D = 12
    p = common.oracle_problem(orc, workloads.paper_run("f2_12d_ray", eval="fp64", seed=2, split=3))
    uid = (3 ** D - 1) // 2
    st, I, m, s, sa = orc.cube(p, 0, uid)
    assert st == 0 and I.max() > 0
    ref = np.std(I * 2.0 ** 600) * 2.0 ** -600
    assert s > 0 and s == pytest.approx(ref, rel=1e-14)
    assert m == pytest.approx(np.mean(I * 2.0 ** 600) * 2.0 ** -600, rel=1e-14)
