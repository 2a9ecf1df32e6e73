"""Exact integrals of the registry's integrands over an axis-aligned box.

Independent of the oracle: these are the textbook antiderivatives, evaluated
with mpmath at 50 significant digits so that alternating sums (the corner-peak
inclusion-exclusion) do not cancel away.  Each takes per-axis arrays lo, hi.
"""
from __future__ import annotations

import itertools

import mpmath as mp

mp.mp.dps = 50


def _m(v):
    return mp.mpf(float(v))


def gauss(sigma, A, mu, lo, hi):
    """A * prod sigma*sqrt(pi/2) * [erf((hi-mu)/(sigma sqrt2)) - erf((lo-mu)/(sigma sqrt2))]."""
    s = _m(sigma)
    r = _m(A)
    for m, a, b in zip(mu, lo, hi):
        k = s * mp.sqrt(2)
        r *= s * mp.sqrt(mp.pi / 2) * (mp.erf((_m(b) - _m(m)) / k) - mp.erf((_m(a) - _m(m)) / k))
    return float(r)


def sin_sum(lo, hi):
    """Im prod_j (e^{i hi_j} - e^{i lo_j}) / i."""
    z = mp.mpc(1)
    for a, b in zip(lo, hi):
        z *= (mp.expj(_m(b)) - mp.expj(_m(a))) / mp.mpc(0, 1)
    return float(z.imag)


def genz_osc(u, c, lo, hi):
    """Re[ e^{2 pi i u} prod_j (e^{i c_j hi_j} - e^{i c_j lo_j}) / (i c_j) ]."""
    z = mp.expj(2 * mp.pi * _m(u))
    for cj, a, b in zip(c, lo, hi):
        cj = _m(cj)
        z *= (mp.expj(cj * _m(b)) - mp.expj(cj * _m(a))) / (mp.mpc(0, 1) * cj)
    return float(z.real)


def genz_ppeak(c, w, lo, hi):
    """prod_j c_j [atan(c_j (hi_j - w_j)) - atan(c_j (lo_j - w_j))]."""
    r = mp.mpf(1)
    for cj, wj, a, b in zip(c, w, lo, hi):
        cj, wj = _m(cj), _m(wj)
        r *= cj * (mp.atan(cj * (_m(b) - wj)) - mp.atan(cj * (_m(a) - wj)))
    return float(r)


def genz_cpeak(c, lo, hi):
    """Integral of (1 + c.x)^-(D+1): D-fold antiderivative, evaluated by
    inclusion-exclusion over the 2^D corners,
    (1 / (D! prod c_j)) sum_v (-1)^{|v|} / (1 + sum_j c_j corner_j(v))."""
    D = len(c)
    cs = [_m(v) for v in c]
    tot = mp.mpf(0)
    for v in itertools.product((0, 1), repeat=D):
        t = mp.mpf(1)
        for j in range(D):
            t += cs[j] * (_m(hi[j]) if v[j] else _m(lo[j]))
        tot += (-1) ** sum(v) / t
    den = mp.factorial(D)
    for cj in cs:
        den *= cj
    return float(tot / den)


def genz_gauss(c, w, lo, hi):
    """prod_j sqrt(pi)/(2 c_j) [erf(c_j (hi_j - w_j)) - erf(c_j (lo_j - w_j))]."""
    r = mp.mpf(1)
    for cj, wj, a, b in zip(c, w, lo, hi):
        cj, wj = _m(cj), _m(wj)
        r *= mp.sqrt(mp.pi) / (2 * cj) * (mp.erf(cj * (_m(b) - wj)) - mp.erf(cj * (_m(a) - wj)))
    return float(r)


def const(A, lo, hi):
    r = _m(A)
    for a, b in zip(lo, hi):
        r *= _m(b) - _m(a)
    return float(r)


def monomial(p, lo, hi):
    """prod_j (hi_j^{p_j+1} - lo_j^{p_j+1}) / (p_j + 1)."""
    r = mp.mpf(1)
    for pj, a, b in zip(p, lo, hi):
        q = int(pj) + 1
        r *= (_m(b) ** q - _m(a) ** q) / q
    return float(r)


def exact(integrand: int, params, lo, hi) -> float:
    """Dispatch on the registry id (0 GAUSS, 1 SIN_SUM, 2 GENZ_OSC, 3 GENZ_PPEAK,
    4 GENZ_CPEAK, 5 GENZ_GAUSS, 6 CONST, 7 MONOMIAL)."""
    D = len(lo)
    p = list(params)
    if integrand == 0:
        return gauss(p[0], p[1], p[2:2 + D], lo, hi)
    if integrand == 1:
        return sin_sum(lo, hi)
    if integrand == 2:
        return genz_osc(p[0], p[1:1 + D], lo, hi)
    if integrand == 3:
        return genz_ppeak(p[:D], p[D:2 * D], lo, hi)
    if integrand == 4:
        return genz_cpeak(p[:D], lo, hi)
    if integrand == 5:
        return genz_gauss(p[:D], p[D:2 * D], lo, hi)
    if integrand == 6:
        return const(p[0], lo, hi)
    if integrand == 7:
        return monomial(p[:D], lo, hi)
    raise ValueError(integrand)


def f1_exact() -> float:
    """The paper's f1 = sin(sum_{i=1..6} x_i) over [0,10]^6 (Sec. 3)."""
    return sin_sum([0.0] * 6, [10.0] * 6)
