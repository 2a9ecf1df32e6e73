"""CPU-side checks of the C ABI: the library loads, exports every function
that include/zmc.h declares, its structs match the binding, and argument
errors are reported without touching the GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1902_07916_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_1902_07916_amd import build
        build.build()
    return _abi.load()


def _declared():
    text = open(os.path.join(ROOT, "include", "zmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(zmc_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    from paper_1902_07916_amd import _abi
    assert set(_abi.EXPORTS) == set(names)


def test_struct_layout(lib):
    from paper_1902_07916_amd import _abi
    for i, T in enumerate((_abi.Result, _abi.Request, _abi.Config, _abi.Trace)):
        assert lib.zmc_struct_size(i) == C.sizeof(T)
    assert lib.zmc_struct_size(9) == -1
    assert b"gfx950" in lib.zmc_version()


def _req(**kw):
    from paper_1902_07916_amd import make_request
    base = dict(integrand="gauss", params=[0.2, 1.0, 0.0, 0.0], lower=-1.0, upper=[1.0, 1.0], divisions=4,
                samples=64, trials=3, max_depth=1, sigma_mult=1.0, seed=1)
    base.update(kw)
    return make_request(**base)


def test_invalid_arguments_are_rejected_before_any_device_call(lib):
    from paper_1902_07916_amd import _abi
    bad = [dict(params=[0.2, 1.0]), dict(divisions=0), dict(samples=0), dict(trials=1), dict(trials=256),
           dict(max_depth=16), dict(max_depth=-1), dict(sigma_mult=-1.0), dict(sigma_mult=float("inf")),
           dict(lower=1.0), dict(upper=[float("nan"), 1.0]), dict(integrand=42), dict(eval=7),
           dict(integrand="monomial", params=[1.5, 2.0]), dict(rtol=-1.0),
           dict(samples=(1 << 33) + 4), dict(divisions=2, max_depth=15, params=[0.2, 1.0] + [0.0] * 2,
                                             lower=[-1.0] * 2, upper=[1.0] * 2, samples=4, trials=2) | {"divisions": 3000000},
           dict(max_cubes_per_level=8),
           # k-way split and threshold scope (Sec. 2.1 variants)
           dict(split=1), dict(split=65), dict(threshold_scope=2), dict(threshold_scope=-1),
           dict(split=64, params=[0.2, 1.0] + [0.0] * 5, lower=[0.0] * 5, upper=[1.0] * 5),
           dict(split=3, max_depth=12, divisions=2, params=[0.2, 1.0] + [0.0] * 5, lower=[0.0] * 5,
                upper=[1.0] * 5)]
    for b in bad:
        r = _req(**b)
        out = _abi.Result()
        rc = lib.zmc_integrate_request(C.byref(r), None, C.byref(out), None)
        assert rc == _abi.EINVAL, b
        assert out.status == _abi.EINVAL
        assert lib.zmc_strerror(rc)


def test_valid_request_without_init(lib):
    from paper_1902_07916_amd import _abi
    out = _abi.Result()
    rc = lib.zmc_integrate_request(C.byref(_req()), None, C.byref(out), None)
    assert rc == _abi.ENOINIT
    t = C.c_uint64()
    assert lib.zmc_submit(C.byref(_req()), C.byref(t)) == _abi.ENOINIT
    assert lib.zmc_poll(1, C.byref(out), 0) == _abi.ENOINIT


def test_init_rejects_bad_config(lib):
    from paper_1902_07916_amd import _abi
    assert lib.zmc_init(None) == _abi.EINVAL
    cfg = _abi.Config()
    cfg.arena = None
    assert lib.zmc_init(C.byref(cfg)) == _abi.EINVAL
    cfg.arena = 256
    cfg.arena_bytes = 1 << 20
    assert lib.zmc_init(C.byref(cfg)) == _abi.EINVAL
    cfg.arena_bytes = 1 << 30
    cfg.arena = 257
    assert lib.zmc_init(C.byref(cfg)) == _abi.EINVAL
    cfg.arena = 256
    for lanes in (-1, 9):
        cfg.serve_lanes = lanes
        assert lib.zmc_init(C.byref(cfg)) == _abi.EINVAL
    cfg.serve_lanes = 0
    cfg.serve_chunk_samples = -2
    assert lib.zmc_init(C.byref(cfg)) == _abi.EINVAL
    cfg.serve_chunk_samples = 0
    cfg.default_eval = 2
    assert lib.zmc_init(C.byref(cfg)) == _abi.EINVAL


def test_integrate_scalar_entry_checks(lib):
    from paper_1902_07916_amd import _abi
    out = _abi.Result()
    lo = (C.c_double * 2)(0.0, 0.0)
    hi = (C.c_double * 2)(1.0, 1.0)
    # sin(sum x) takes no params; the Gaussian takes 2 + D, derived from dim
    rc = lib.zmc_integrate(_abi.SIN_SUM, None, 2, lo, hi, 2, 16, 3, 1, 1.0, 1, None, C.byref(out))
    assert rc == _abi.ENOINIT
    prm = (C.c_double * 4)(0.2, 1.0, 0.5, 0.5)
    rc = lib.zmc_integrate(_abi.GAUSS, prm, 2, lo, hi, 2, 16, 3, 1, 1.0, 1, None, C.byref(out))
    assert rc == _abi.ENOINIT
    rc = lib.zmc_integrate(_abi.GAUSS, None, 2, lo, hi, 2, 16, 3, 1, 1.0, 1, None, C.byref(out))
    assert rc == _abi.EINVAL
    rc = lib.zmc_integrate(_abi.SIN_SUM, None, 2, None, hi, 2, 16, 3, 1, 1.0, 1, None, C.byref(out))
    assert rc == _abi.EINVAL
    rc = lib.zmc_integrate(42, None, 2, lo, hi, 2, 16, 3, 1, 1.0, 1, None, C.byref(out))
    assert rc == _abi.EINVAL and out.status == _abi.EINVAL


def test_integrate_has_the_documented_signature():
    """zmc_integrate takes exactly (integrand_id, params, dim, lower, upper,
    divisions_per_axis, samples_per_cube, trials, max_depth, sigma_mult,
    seed, stream, out): the parameter count is derived from the integrand
    and the evaluation mode comes from the configuration."""
    text = open(os.path.join(ROOT, "include", "zmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    decl = re.search(r"int zmc_integrate\((.*?)\);", text, flags=re.S).group(1)
    names = [re.split(r"[\s*]+", a.strip())[-1] for a in decl.split(",")]
    assert names == ["integrand_id", "params", "dim", "lower", "upper", "divisions_per_axis", "samples_per_cube",
                     "trials", "max_depth", "sigma_mult", "seed", "stream", "out"]
    assert re.search(r"int32_t default_eval;", text)


def test_workloads_are_deterministic():
    from paper_1902_07916_amd import workloads as W
    a = W.genz_batch(n=32)
    b = W.genz_batch(n=32)
    assert a == b
    assert all(2 <= len(r["lower"]) <= 12 and r["divisions"] ** len(r["lower"]) <= 100_000 for r in a)
    s = W.serving_stream(duration=2.0)
    assert 300 < len(s) < 500 and all(3 <= len(r["lower"]) <= 12 for _, r in s)
    assert all(1e-5 <= r["rtol"] <= 1e-3 for _, r in s)
    assert all(r["divisions"] ** len(r["lower"]) <= 4096 for _, r in s)


def test_split_limits_agree_with_oracle(lib, orc):
    """The library accepts exactly the (D, split, divisions, depth) shapes the
    oracle accepts: children per split <= 2^24 and every uid below 2^64."""
    from paper_1902_07916_amd import _abi, make_request
    for D in (1, 2, 3, 5, 8, 12):
        for b in (0, 2, 3, 5, 16, 64):
            for d in (1, 3, 7):
                for dep in (0, 1, 4, 7, 9, 15):
                    prm = [0.2, 1.0] + [0.0] * D
                    r = make_request("gauss", prm, [0.0] * D, [1.0] * D, d, 4, 3, dep, 1.0, 1, split=b)
                    out = _abi.Result()
                    rc = lib.zmc_integrate_request(C.byref(r), None, C.byref(out), None)
                    p = orc.problem(0, D, [0.0] * D, [1.0] * D, d, 4, 3, dep, 1.0, 1, params=prm, split=b or 2)
                    # the oracle checks d^D against the level cap when a run starts
                    ok = orc.validate(p) == 0 and d ** D <= (1 << 24)
                    assert (rc == _abi.ENOINIT) == ok, (D, b, d, dep, rc)
                    assert rc in (_abi.ENOINIT, _abi.EINVAL)


def _step_bytes(n, n_next, trials, nch, kids, scope, level):
    """Device bytes the level driver holds while stepping a level of n cubes
    whose next level has n_next cubes: the current uid list, the partial sums
    (one 16-byte pair per (cube, trial, chunk)), m, s, the selection bytes,
    the 96-byte tile records (one per 1024 cubes), the per-parent thresholds
    (one per sibling group) and the next uid list, each rounded to 256 bytes."""
    r = lambda b: (b + 255) // 256 * 256  # noqa: E731
    groups = n // kids if (scope == 1 and level > 0 and n > kids) else 0
    return (r(8 * n) + r(16 * trials * nch * n) + 2 * r(8 * n) + r(n) + r(96 * -(-n // 1024)) + r(8 * groups)
            + r(8 * n_next))


def test_request_bytes_bounds_every_level(lib):
    """The admission reservation covers every level of the worst-case tree
    (Cantelli's bound on the selections, the level cap), for both threshold
    scopes and small D, where the per-parent thresholds weigh most."""
    import math

    from paper_1902_07916_amd import _abi, make_request
    checked = 0
    for D in (1, 2, 3):
        for scope in (0, 1):
            for split in (0, 3):
                for sigma in (0.0, 0.5, 1.0, 5.0):
                    big = {1: 200000, 2: 447, 3: 58}[D]  # ~2e5 roots: the per-cube terms dominate
                    for d, N, n1, depth in ((5, 1000, 2, 4), (big, 4096, 3, 3), (big, 128, 5, 2)):
                        prm = [0.2, 1.0] + [0.0] * D
                        q = make_request("gauss", prm, [0.0] * D, [1.0] * D, d, N, n1, depth, sigma, 1,
                                         split=split, threshold_scope=scope)
                        got = C.c_uint64()
                        assert lib.zmc_request_bytes(C.byref(q), C.byref(got)) == 0
                        kids = (split or 2) ** D
                        groups = min(-(-N // 256), 32)
                        nch = -(-N // (256 * groups))
                        n = d ** D
                        sizes = [n]
                        for _ in range(depth):
                            nsel = n - 1 if sigma == 0 else math.floor(n / (1 + sigma * sigma))
                            nn = nsel * kids
                            if nn > (1 << 24) or nn == 0:
                                break
                            sizes.append(nn)
                            n = nn
                        need = max(_step_bytes(a, b, n1, nch, kids, scope, l)
                                   for l, (a, b) in enumerate(zip(sizes, sizes[1:] + [0])))
                        assert got.value >= need, (D, scope, split, sigma, d, got.value, need)
                        checked += 1
    assert checked == 144
    bad = make_request("gauss", [0.2], [0.0], [1.0], 2, 16, 3, 1, 1.0, 1)
    assert lib.zmc_request_bytes(C.byref(bad), C.byref(C.c_uint64())) == _abi.EINVAL
