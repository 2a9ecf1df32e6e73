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


# Unit roundoff of FP64.
U64 = 2.0 ** -53
# Bound on |I_t(GPU) - I_t(oracle)| for one (cube, trial), relative to the
# trial's estimate of the cube's integral of |f|, V * sum |f| / N, in FP32
# evaluation: the cube-relative FP32 arguments and the hardware exp2 / rcp /
# the polynomial sine are each within a few FP32 ulps of the FP64 value at
# every point (measured maximum over every traced parity case: see the
# design notes), so a trial's sum is too.
FP32_TRIAL_TOL = 2e-5


# Absolute floor of |ds| for values near the subnormal range (see compare_tree).
S_FLOOR = 2.0 ** -532


def trial_tol(eval_, N, w=None, level=0):
    """Per-trial bound relative to V * sum |f| / N from the summation: both
    sides sum the same N values in different orders, and a recursive sum is
    within (N - 1) u of the sum of |f| (u = 2^-53); FP32: FP32_TRIAL_TOL,
    measured, covering the evaluation too, or the product peak's argument
    conditioning at this level where that is larger (fp32_ppeak_error)."""
    if eval_ == "fp64":
        return (2 * N + 8) * U64
    if w is not None and w["integrand"] == 3:
        return max(FP32_TRIAL_TOL, fp32_ppeak_error(w, level))
    return FP32_TRIAL_TOL


def fp32_ppeak_error(w, level):
    """Relative error bound of one FP32 product-peak value at a level.

    The FP32 form evaluates prod 1 / (1 + u_i^2) with u_i = m_i v_i + a_i,
    where m_i = c_i h_i and a_i (the cube's offset from the peak, scaled
    by c_i) are rounded to FP32 once per cube and v_i is exact.  Then
    |du_i| <= (|a_i| + |m_i| + |u_i|) 2^-24 <= (2 |u_i| + 2 |m_i|) 2^-24
    (|a_i| <= |u_i| + |m_i| because v_i lies in (0, 1)), and the relative
    change of 1 / (1 + u^2) is at most 2 |u| |du| / (1 + u^2), which with
    |u| / (1 + u^2) <= 1/2 gives (4 + 2 |m_i|) 2^-24 per axis.  Add one
    rounding for each fma, product and the reciprocal (2 D + 4).  The
    width h_i at the level is the root width over split^level.  A sharp
    peak (c h >> 1) is where this exceeds the measured FP32 bound."""
    D = len(w["lower"])
    c = np.abs(np.asarray(w["params"][:D], float))
    h = (np.asarray(w["upper"], float) - np.asarray(w["lower"], float)) / w["divisions"]
    h = h / float((w.get("split", 0) or 2) ** level)
    return 2.0 ** -24 * (float(np.sum(4.0 + 2.0 * c * h)) + 2 * D + 4)


def fp64_point_error(w):
    """Bound on the difference of two FP64 evaluations of the same f at the
    same point (the library's and libm's), as |df| <= rho |f| + alpha.

    Each side rounds the transcendental's argument after a few operations,
    and a correctly rounded (or few-ulp) function of an argument off by
    |arg| c u is off by the argument's error times its derivative: for exp,
    a relative |arg| c u; for sin / cos, an absolute |arg| c u.  c = D + 4
    covers the D + 2 roundings of the argument's sum and product and a 2-ulp
    function on either side.  Rational / power families: one rounding per
    operation.  Gaussians also scale a possibly subnormal exp by A, whose
    absolute error is then |A| 2^-1074 per rounding (alpha).  |arg| is
    bounded over the whole domain."""
    import math
    D = len(w["lower"])
    lo = np.asarray(w["lower"], float)
    hi = np.asarray(w["upper"], float)
    prm = np.asarray(w["params"], float)
    c = D + 4
    f = w["integrand"]
    if f == 0:    # A exp(-|x - mu|^2 / (2 sigma^2))
        mu = prm[2:2 + D]
        q = float(np.sum(np.maximum((lo - mu) ** 2, (hi - mu) ** 2)))
        return q / (2 * prm[0] ** 2) * c * U64 + 4 * U64, 16 * abs(prm[1]) * 2.0 ** -1074
    if f == 1:    # sin(sum x)
        return 4 * U64, float(np.sum(np.maximum(abs(lo), abs(hi)))) * c * U64
    if f == 2:    # cos(2 pi u + c.x)
        cc = prm[1:1 + D]
        return 4 * U64, (2 * math.pi * abs(prm[0]) + float(np.sum(abs(cc) * np.maximum(abs(lo), abs(hi))))) * c * U64
    if f == 3:    # prod 1 / (c^-2 + (x - w)^2)
        return 8 * D * U64, 0.0
    if f == 4:    # (1 + c.x)^-(D+1)
        return 4 * (D + 2) ** 2 * U64, 0.0
    if f == 5:    # exp(-sum c^2 (x - w)^2)
        cc, ww = prm[:D], prm[D:2 * D]
        q = float(np.sum(cc ** 2 * np.maximum((lo - ww) ** 2, (hi - ww) ** 2)))
        return q * c * U64 + 4 * U64, 16 * 2.0 ** -1074
    if f == 6:    # A
        return 0.0, 0.0
    if f == 7:    # prod x^p
        return 4 * (float(np.sum(prm[:D])) + D) * U64, 0.0
    return 64 * U64, 0.0


def compare_tree(orc, w, r, eps, tol, report=None):
    """Whole-tree comparison of a traced GPU run with the oracle, which
    replays the GPU's decisions inside the margin band.

    Per level: the cube list bit-exact; per (cube, trial) |dI_t| within
    trial_tol times the trial's estimate of the integral of |f| (bounded by
    n1 times the oracle's per-cube sa); per cube |dm| and |ds| within
    max_t |dI_t| plus a few ulps of the largest trial value (the mean is
    1-Lipschitz and the population std a norm of the centred trial vector,
    so neither moves by more than the largest trial difference); the level
    threshold within (1 + sigma_mult) max_c |ds_c| (mean and population std
    of the s are 1-Lipschitz in the largest difference) and, in FP64, 1e-12
    relative; each selection the strict rule against its own cube's
    threshold outside the margin band and equal to the oracle's there.
    Totals: integral within tol relative (or tol times the oracle's integral
    of |f| where the integral is near 0), std within tol relative."""
    p = oracle_problem(orc, w)
    replay = [(L["uid"], L["sel"], L["uid_hi"]) for L in r.trace]
    o = orc.integrate(p, replay=replay, band_eps=eps)
    assert o.status == 0 and r.status == 0
    assert len(o.levels) == r.levels_run
    eval_ = w.get("eval", "fp64")
    N, n1 = int(w["samples"]), int(w["trials"])
    rho, alpha = fp64_point_error(w) if eval_ == "fp64" else (0.0, 0.0)
    stats = dict(dI=0.0, ds=0.0, dthr=0.0)
    for l, (Lo, Lg) in enumerate(zip(o.levels, r.trace)):
        assert Lg["n"] == Lo.n
        assert len(Lg["uid"]) == Lg["n"], "trace capacity too small"
        assert np.array_equal(Lg["uid"], Lo.uid), "level %d list differs" % l
        assert np.array_equal(Lg["uid_hi"], Lo.uid_hi), "level %d list differs (id bits above 64)" % l
        V = orc.bounds(p, l, int(Lo.uid[0]) | (int(Lo.uid_hi[0]) << 64))[2]
        Ig = V * (np.asarray(Lg["S1"]) / N)
        dI = np.abs(Ig - Lo.I).max(axis=1)
        scale = n1 * Lo.sa
        Imax = np.abs(Lo.I).max(axis=1)
        with np.errstate(divide="ignore", invalid="ignore"):
            stats["dI"] = max(stats["dI"], float(np.nanmax(np.where(scale > 0, dI / scale, 0.0))))
        bound_I = (trial_tol(eval_, N, w, l) + rho) * scale + V * alpha
        worst = int(np.argmax(dI - bound_I))
        assert np.all(dI <= bound_I), ("level %d trial sums" % l, worst, dI[worst], bound_I[worst], scale[worst])
        slack = 4 * (n1 + 2) * U64 * Imax
        dm = np.abs(np.asarray(Lg["m"]) - Lo.m)
        ds = np.abs(np.asarray(Lg["s"]) - Lo.s)
        assert np.all(dm <= dI + slack), "level %d m" % l
        # s = sqrt(sum (I_t - m)^2 / n1), the deviations scaled by a power of
        # two first, so their squares do not underflow; trial values and
        # deviations below the normal range still carry absolute roundings of
        # 2^-1074, which the relative slack does not cover.  S_FLOOR bounds
        # them generously: it is the bound for unscaled squares, whose
        # rounding to multiples of 2^-1074 gives s an absolute error of at
        # most sqrt(2 n1 2^-1074) < 2^-532.
        assert np.all(ds <= dI + slack + S_FLOOR), "level %d s" % l
        with np.errstate(divide="ignore", invalid="ignore"):
            stats["ds"] = max(stats["ds"], float(np.nanmax(np.where(dI + slack + S_FLOOR > 0,
                                                                    ds / (dI + slack + S_FLOOR), 0.0))))
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
                dthr = abs(r.thr_per_level[l] - Lo.thr)
                bound = (1 + w["sigma_mult"]) * float(ds.max()) + 4 * (Lo.n + 2) * U64 * abs(Lo.thr)
                assert dthr <= bound, ("level %d threshold" % l, dthr, bound)
                if eval_ == "fp64":
                    assert rel(r.thr_per_level[l], Lo.thr) < 1e-12
                stats["dthr"] = max(stats["dthr"], rel(r.thr_per_level[l], Lo.thr))
    assert rel(r.integral, o.integral) < tol or abs(r.integral - o.integral) < tol * o.sum_abs
    assert rel(r.std, o.std) < tol or (r.std == 0.0 and o.std == 0.0)
    stats.update(integral=rel(r.integral, o.integral), std=rel(r.std, o.std))
    print("compare_tree %s: max dI/(n1 sa) %.3g, max ds/bound %.3g, thr rel %.3g, integral rel %.3g, std rel %.3g"
          % (eval_, stats["dI"], stats["ds"], stats["dthr"], stats["integral"], stats["std"]))
    if report is not None:
        report.update(stats)
    return o


def check_levels_sampled(orc, w, r, n_sample, m_tol, m_floor=0.0, seed=0):
    """Parity of a traced run too large for the whole oracle tree.  Per level:
    sampled cubes (first, last, n_sample random ones, every selected cube)
    recomputed by the oracle one by one (m, s within m_tol times the cube's
    integral of |f| estimate, plus m_floor); the threshold recomputed by the
    oracle over the GPU's own s (within 4 (n + 2) u, at least 1e-12, for n
    cubes); the selection the strict rule against it (no cube that close to
    it); the next list the children of
    the selected cubes in order; totals the sums of the accepted m and s^2.
    m_floor: absolute slack for values FP32 cannot represent."""
    import math
    p = oracle_problem(orc, w)
    D = len(w["lower"])
    b = w.get("split", 0) or 2
    kids_n = b ** D
    rng = np.random.default_rng(seed)
    acc_m, acc_s2 = [], []
    for l, L in enumerate(r.trace):
        assert len(L["uid"]) == L["n"] == r.cubes_per_level[l]
        sel = L["sel"].astype(bool)
        last = not (l < w["max_depth"] and l + 1 < len(r.trace))
        idx = [0, L["n"] - 1] + list(rng.integers(0, L["n"], n_sample))
        if not last:
            idx += list(np.nonzero(sel)[0][:64])
        for i in np.unique(idx):
            st, I, m, s, sa = orc.cube(p, l, int(L["uid"][i]) | (int(L["uid_hi"][i]) << 64))
            assert st == 0
            assert abs(L["m"][i] - m) <= m_tol * sa + m_floor, (l, i, L["m"][i], m, sa)
            assert abs(L["s"][i] - s) <= m_tol * sa * 10 + 1e-9 * s + m_floor, (l, i, L["s"][i], s)
        if not last:
            # the same threshold formula over the same n values, summed in
            # another order: each of the two sums is within (n - 1) u of
            # exact on either side, so thr agrees to 4 (n + 2) u relative
            thr, mu, sd = orc.threshold(L["s"], w["sigma_mult"])
            thr_eps = max(1e-12, 4 * (L["n"] + 2) * U64)
            nz = int(np.count_nonzero(L["s"]))
            assert rel(r.thr_per_level[l], thr) < thr_eps, ("level %d threshold" % l, r.thr_per_level[l], thr, mu,
                                                           sd, nz, float(np.max(L["s"])))
            band = margin_band_ok(L["s"], L["sel"], thr, thr_eps)
            assert len(band) == 0, "cubes within %.3g of the threshold: %s" % (thr_eps, band)
            assert int(sel.sum()) == r.selected_per_level[l]
            parents = L["uid"][sel]
            parents_hi = L["uid_hi"][sel]
            # ids below 2^64: children as uint64 arithmetic (wraps past 2^64,
            # compared with the low bits); every parent: the oracle's children
            kids = (parents[:, None] * np.uint64(kids_n) + np.arange(kids_n, dtype=np.uint64)[None, :]).ravel()
            assert np.array_equal(r.trace[l + 1]["uid"], kids)
            picks = range(len(parents)) if len(parents) <= 8 else rng.integers(0, len(parents), 8)
            for j in picks:
                clo, chi = orc.children_w(int(parents[j]) | (int(parents_hi[j]) << 64), D, b)
                assert np.array_equal(clo, kids[j * kids_n:(j + 1) * kids_n])
                assert np.array_equal(chi, r.trace[l + 1]["uid_hi"][j * kids_n:(j + 1) * kids_n])
            keep = ~sel
        else:
            keep = np.ones(L["n"], bool)
        acc_m.append(L["m"][keep])
        acc_s2.append(L["s"][keep] ** 2)
    M = math.fsum(np.concatenate(acc_m))
    S2 = math.fsum(np.concatenate(acc_s2))
    assert rel(r.integral, M) < 1e-10 or abs(r.integral - M) < 1e-12 * float(np.abs(np.concatenate(acc_m)).sum())
    assert rel(r.std, math.sqrt(S2)) < 1e-10 or (r.std == 0.0 and S2 == 0.0)
