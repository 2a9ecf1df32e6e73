"""User-defined integrands: a body compiled at run time (hipRTC) on the GPU
side and with g++ on the oracle side.  CPU tests cover registration and the
oracle hook; GPU tests compare the run-time kernels with the precompiled
registry (bit for bit where the arithmetic is the same) and with the oracle."""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import closed_forms as cf  # noqa: E402
from common import oracle_problem, rel  # noqa: E402

SIN_BODY = "real t = 0; for (int i = 0; i < D; ++i) t += x[i]; return sin(t);"
# a Gaussian with per-axis width p[0] and centre p[1] (the same for all axes)
GAUSS_BODY = "real q = 0; for (int i = 0; i < D; ++i) { real d = x[i] - (real)p[1]; q += d * d; } " \
             "return exp(-q / (real)(2 * p[0] * p[0]));"


@pytest.fixture(scope="module")
def zmc():
    import paper_1902_07916_amd as z
    from paper_1902_07916_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("library not built")
    return z


def test_register_and_errors(zmc):
    i = zmc.register_integrand(SIN_BODY, 0)
    assert i >= 100
    j = zmc.register_integrand(GAUSS_BODY, 2)
    assert j > i
    with pytest.raises(zmc.ZmcError) as e:
        zmc.register_integrand("return sin(x[0]) +* p[0];", 1)
    assert e.value.code == -1 and "error" in str(e.value)
    with pytest.raises(zmc.ZmcError):
        zmc.register_integrand(SIN_BODY, 99)


def test_oracle_user_hook_reproduces_registry(orc):
    orc.set_user(120, SIN_BODY, 0)
    a = orc.integrate(orc.problem(orc.SIN_SUM, 3, 0.0, 2.0, 3, 256, 4, 1, 1.0, 5))
    b = orc.integrate(orc.problem(120, 3, 0.0, 2.0, 3, 256, 4, 1, 1.0, 5))
    assert a.integral == b.integral and a.std == b.std
    assert all(np.array_equal(x.uid, y.uid) for x, y in zip(a.levels, b.levels))


def test_oracle_user_gauss_closed_form(orc):
    orc.set_user(121, GAUSS_BODY, 2)
    p = orc.problem(121, 3, [0.0] * 3, [1.0] * 3, 3, 1024, 5, 2, 1.0, 3, params=[0.2, 0.4])
    r = orc.integrate(p)
    exact = cf.gauss(0.2, 1.0, [0.4] * 3, [0.0] * 3, [1.0] * 3)
    assert abs(r.integral - exact) <= 5 * r.stderr


@pytest.mark.gpu
def test_user_sin_bitwise_equals_registry_fp64(zmc):
    from paper_1902_07916_amd import Integrator, workloads as W
    zi = Integrator(arena_bytes=4 << 30)
    try:
        uid = zmc.register_integrand(SIN_BODY, 0)
        w = W.sin6d(eval="fp64", samples=2048, divisions=4, max_depth=2)
        a = zi.integrate(**w)
        b = zi.integrate(**dict(w, integrand=uid))
        assert a.integral == b.integral and a.std == b.std and a.cubes_per_level == b.cubes_per_level
    finally:
        zi.close()


@pytest.mark.gpu
@pytest.mark.parametrize("eval_,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_user_gauss_matches_oracle(zmc, orc, eval_, tol):
    from paper_1902_07916_amd import Integrator
    zi = Integrator(arena_bytes=4 << 30)
    try:
        uid = zmc.register_integrand(GAUSS_BODY, 2)
        orc.set_user(uid, GAUSS_BODY, 2)
        w = dict(integrand=uid, params=[0.2, 0.4], lower=[0.0] * 4, upper=[1.0] * 4, divisions=3, samples=3001,
                 trials=4, max_depth=2, sigma_mult=1.0, seed=9, eval=eval_)
        r = zi.integrate(**w, trace=True)
        o = orc.integrate(oracle_problem(orc, w), replay=[(L["uid"], L["sel"]) for L in r.trace],
                          band_eps=1e-9 if eval_ == "fp64" else 1e-4)
        assert [L.n for L in o.levels] == r.cubes_per_level
        assert rel(r.integral, o.integral) < tol
        assert rel(r.std, o.std) < 10 * tol
    finally:
        zi.close()
