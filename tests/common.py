"""Helpers shared by the GPU parity tests: translate a workload dict into
the oracle's problem and into a library request, and compare level traces."""
import numpy as np


def oracle_problem(orc, w):
    D = len(w["lower"])
    return orc.problem(w["integrand"], D, w["lower"], w["upper"], w["divisions"], w["samples"], w["trials"],
                       w["max_depth"], w["sigma_mult"], w["seed"], params=w["params"], rtol=w.get("rtol", 0.0),
                       max_cubes_per_level=w.get("max_cubes_per_level", 0) or (1 << 24),
                       split=w.get("split", 0) or 2, scope=w.get("scope", 0))


def request(w):
    from paper_1902_07916_amd import request_from_dict
    return request_from_dict(w)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def margin_band_ok(s_gpu, sel_gpu, thr, eps):
    """Decisions taken on the GPU's own s against thr: outside the band of
    relative half-width eps they must be the strict rule; inside either is
    acceptable.  Returns the indices inside the band."""
    s_gpu = np.asarray(s_gpu)
    sel_gpu = np.asarray(sel_gpu).astype(bool)
    margin = np.abs(s_gpu - thr) / thr
    out = margin > eps
    assert np.array_equal(sel_gpu[out], (s_gpu > thr)[out])
    return np.nonzero(~out)[0]


def cube_thresholds(orc, w, level, s):
    """Each cube's threshold from a level's s: one per level (scope 0, or the
    roots), else one per group of split^D siblings (per-parent scope)."""
    D = len(w["lower"])
    kids = (w.get("split", 0) or 2) ** D
    s = np.asarray(s)
    if w.get("scope", 0) == 1 and level > 0 and len(s) > kids:
        assert len(s) % kids == 0
        out = np.empty(len(s))
        for g in range(0, len(s), kids):
            out[g:g + kids] = orc.threshold(s[g:g + kids], w["sigma_mult"])[0]
        return out
    return np.full(len(s), orc.threshold(s, w["sigma_mult"])[0])


def compare_tree(orc, w, r, eps, tol):
    """Whole-tree comparison of a traced GPU run with the oracle, which
    replays the GPU's decisions inside the margin band: lists bit-exact, m and
    s within tol, each selection against its own cube's threshold outside the
    band, totals within tol."""
    p = oracle_problem(orc, w)
    replay = [(L["uid"], L["sel"]) for L in r.trace]
    o = orc.integrate(p, replay=replay, band_eps=eps)
    assert o.status == 0 and r.status == 0
    assert len(o.levels) == r.levels_run
    for l, (Lo, Lg) in enumerate(zip(o.levels, r.trace)):
        assert Lg["n"] == Lo.n
        assert len(Lg["uid"]) == Lg["n"], "trace capacity too small"
        assert np.array_equal(Lg["uid"], Lo.uid), "level %d list differs" % l
        np.testing.assert_allclose(Lg["m"], Lo.m, rtol=tol, atol=tol * np.abs(Lo.m).max())
        s_scale = max(np.abs(Lo.s).max(), 1e-12 * np.abs(Lo.m).max())
        np.testing.assert_allclose(Lg["s"], Lo.s, rtol=max(tol, 1e-9) * 100, atol=tol * s_scale)
        if l < w["max_depth"]:
            thr = cube_thresholds(orc, w, l, Lo.s)
            sel = np.asarray(Lg["sel"]).astype(bool)
            with np.errstate(divide="ignore", invalid="ignore"):
                margin = np.abs(Lg["s"] - thr) / thr
            out = ~(margin <= eps)
            assert np.array_equal(sel[out], (Lg["s"] > thr)[out]), "level %d selection" % l
            # outside the band the oracle decided the same (replay only inside)
            assert np.array_equal(sel[out], Lo.sel[out].astype(bool))
            if np.isnan(Lo.thr):
                assert np.isnan(r.thr_per_level[l])
            else:
                assert rel(r.thr_per_level[l], Lo.thr) < max(tol, 1e-12) * 100
    assert rel(r.integral, o.integral) < tol or abs(r.integral - o.integral) < tol * o.sum_abs
    assert rel(r.std, o.std) < tol * 10
    return o
