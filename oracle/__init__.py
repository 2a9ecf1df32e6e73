"""CPU oracle for the ZMCintegral method (arXiv:1902.07916, Sec. 2.1).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product package never imports this
module and this module imports nothing from the product package.

The arithmetic lives in ``zmc_oracle.c`` (plain single-threaded FP64 C, built
with ``-ffp-contract=off`` and no fast-math); this file only marshals arguments
through ctypes and exposes the runs as numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "zmc_oracle.c")
BUILD_DIR = os.path.join(HERE, "_build")
LIB_PATH = os.path.join(BUILD_DIR, "libzmc_oracle.so")

MAX_DIM = 16
MAX_LEVELS = 16
MAX_PARAMS = 2 * MAX_DIM + 2

GAUSS, SIN_SUM, GENZ_OSC, GENZ_PPEAK, GENZ_CPEAK, GENZ_GAUSS, CONST, MONOMIAL = range(8)
OK, EINVAL, ENOMEM, ENONFINITE = 0, -1, -2, -3
F_TRUNCATED, F_RTOL_MET = 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/_build`` and return the path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Problem(C.Structure):
    _fields_ = [
        ("integrand", C.c_int32), ("dim", C.c_int32), ("divisions", C.c_int32),
        ("trials", C.c_int32), ("max_depth", C.c_int32), ("n_params", C.c_int32),
        ("split", C.c_int32), ("scope", C.c_int32),
        ("samples", C.c_int64), ("max_cubes_per_level", C.c_int64),
        ("sigma_mult", C.c_double), ("rtol", C.c_double), ("seed", C.c_uint64),
        ("lower", C.c_double * MAX_DIM), ("upper", C.c_double * MAX_DIM),
        ("params", C.c_double * MAX_PARAMS),
    ]


class Replay(C.Structure):
    _fields_ = [
        ("n_levels", C.c_int32),
        ("n", C.c_int64 * MAX_LEVELS),
        ("uid", C.POINTER(C.c_uint64) * MAX_LEVELS),
        ("uid_hi", C.POINTER(C.c_uint32) * MAX_LEVELS),
        ("sel", C.POINTER(C.c_uint8) * MAX_LEVELS),
    ]


ID_BITS = 84  # cube ids: bits 0..63 in uid, 64..83 in uid_hi


def _split_id(uid):
    uid = int(uid)
    if uid < 0 or uid >> ID_BITS:
        raise ValueError("cube id out of range")
    return uid & ((1 << 64) - 1), uid >> 64


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = LIB_PATH if os.path.exists(LIB_PATH) else build()
        L = C.CDLL(path)
        P = C.POINTER(Problem)
        L.oracle_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.oracle_uniform.argtypes = [C.c_uint32]
        L.oracle_uniform.restype = C.c_double
        L.oracle_word.argtypes = [C.c_uint64, C.c_uint64, C.c_int, C.c_int, C.c_int, C.c_int64, C.c_int]
        L.oracle_word.restype = C.c_uint32
        L.oracle_word_w.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_int, C.c_int, C.c_int, C.c_int64,
                                    C.c_int]
        L.oracle_word_w.restype = C.c_uint32
        L.oracle_cube_lattice_w.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint64, C.c_uint32,
                                            C.POINTER(C.c_uint64)]
        L.oracle_cube_bounds_w.argtypes = [P, C.c_int, C.c_uint64, C.c_uint32, C.POINTER(C.c_double),
                                           C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_sample_x_w.argtypes = [P, C.c_int, C.c_uint64, C.c_uint32, C.c_int, C.c_int64,
                                        C.POINTER(C.c_double)]
        L.oracle_cube_trial_w.argtypes = [P, C.c_int, C.c_uint64, C.c_uint32, C.c_int, C.POINTER(C.c_double),
                                          C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_cube_w.argtypes = [P, C.c_int, C.c_uint64, C.c_uint32, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_children_w.argtypes = [C.c_uint64, C.c_uint32, C.c_int, C.c_int, C.POINTER(C.c_uint64),
                                        C.POINTER(C.c_uint32)]
        L.oracle_cube_lattice.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint64, C.POINTER(C.c_uint64)]
        L.oracle_cube_bounds.argtypes = [P, C.c_int, C.c_uint64, C.POINTER(C.c_double),
                                         C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_n_params.argtypes = [C.c_int, C.c_int]
        L.oracle_f.argtypes = [C.c_int, C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_double)]
        L.oracle_f.restype = C.c_double
        L.oracle_sample_x.argtypes = [P, C.c_int, C.c_uint64, C.c_int, C.c_int64, C.POINTER(C.c_double)]
        L.oracle_cube_trial.argtypes = [P, C.c_int, C.c_uint64, C.c_int, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_cube.argtypes = [P, C.c_int, C.c_uint64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_threshold.argtypes = [C.POINTER(C.c_double), C.c_int64, C.c_double,
                                       C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_threshold.restype = C.c_double
        L.oracle_children.argtypes = [C.c_uint64, C.c_int, C.c_int, C.POINTER(C.c_uint64)]
        L.oracle_validate.argtypes = [P]
        L.oracle_integrate.argtypes = [P, C.POINTER(Replay), C.c_double]
        L.oracle_integrate.restype = C.c_void_p
        L.oracle_free.argtypes = [C.c_void_p]
        for name in ("oracle_run_status", "oracle_run_flags", "oracle_run_levels"):
            getattr(L, name).argtypes = [C.c_void_p]
        L.oracle_run_totals.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]
        L.oracle_level_n.argtypes = [C.c_void_p, C.c_int]
        L.oracle_level_n.restype = C.c_int64
        for name, t in (("oracle_level_uid", C.c_uint64), ("oracle_level_uid_hi", C.c_uint32),
                        ("oracle_level_m", C.c_double),
                        ("oracle_level_s", C.c_double), ("oracle_level_I", C.c_double),
                        ("oracle_level_sa", C.c_double), ("oracle_level_sel", C.c_uint8)):
            f = getattr(L, name)
            f.argtypes = [C.c_void_p, C.c_int]
            f.restype = C.POINTER(t)
        L.oracle_level_stats.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.oracle_set_user.argtypes = [C.c_int, C.c_void_p, C.c_int]
        if L.oracle_sizeof_problem() != C.sizeof(Problem):
            raise RuntimeError("oracle_problem layout mismatch")
        _lib = L
    return _lib


def problem(integrand, dim, lower, upper, divisions, samples, trials, max_depth, sigma_mult, seed,
            params=(), rtol=0.0, max_cubes_per_level=1 << 24, split=2, scope=0) -> Problem:
    p = Problem()
    p.integrand, p.dim, p.divisions = int(integrand), int(dim), int(divisions)
    p.split, p.scope = int(split), int(scope)
    p.trials, p.max_depth, p.n_params = int(trials), int(max_depth), len(params)
    p.samples, p.max_cubes_per_level = int(samples), int(max_cubes_per_level)
    p.sigma_mult, p.rtol, p.seed = float(sigma_mult), float(rtol), int(seed) & ((1 << 64) - 1)
    nd = max(0, min(int(dim), MAX_DIM))
    lower = np.broadcast_to(np.asarray(lower, dtype=np.float64), (nd,))
    upper = np.broadcast_to(np.asarray(upper, dtype=np.float64), (nd,))
    for i in range(nd):
        p.lower[i] = float(lower[i])
        p.upper[i] = float(upper[i])
    if len(params) > MAX_PARAMS:
        raise ValueError("too many params")
    for j, v in enumerate(params):
        p.params[j] = float(v)
    return p


_user_libs = []


def build_user(body: str) -> str:
    """Compile a user integrand body with g++ into a shared library exposing
    double zmc_user_f(const double* x, const double* p, int D), the same body
    the GPU path compiles (there `real` is double or float)."""
    import hashlib
    os.makedirs(BUILD_DIR, exist_ok=True)
    tag = hashlib.sha256(body.encode()).hexdigest()[:16]
    src = os.path.join(BUILD_DIR, "user_%s.cpp" % tag)
    so = os.path.join(BUILD_DIR, "user_%s.so" % tag)
    if not os.path.exists(so):
        with open(src, "w") as fh:
            fh.write("#include <cmath>\nusing namespace std;\n"
                     "extern \"C\" double zmc_user_f(const double* x, const double* p, int D)\n"
                     "{\n    using real = double;\n    (void)p;\n    (void)D;\n" + body + "\n}\n")
        tmp = so + ".tmp%d" % os.getpid()
        subprocess.run(["g++", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", tmp, src], check=True)
        os.replace(tmp, so)
    return so


def set_user(integrand_id: int, body: str, n_params: int) -> None:
    """Register a user integrand with the oracle under the same id the GPU
    library returned."""
    lib_u = C.CDLL(build_user(body))
    _user_libs.append(lib_u)
    fn = C.cast(lib_u.zmc_user_f, C.c_void_p).value
    if lib().oracle_set_user(int(integrand_id), fn, int(n_params)) != 0:
        raise ValueError("oracle_set_user failed")


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return tuple(o)


def uniform(w: int) -> float:
    return lib().oracle_uniform(int(w) & 0xFFFFFFFF)


def word(seed, uid, level, trial, dim, s, i) -> int:
    """uid: a cube id of up to 84 bits (a Python int)."""
    lo, hi = _split_id(uid)
    return lib().oracle_word_w(int(seed), lo, hi, int(level), int(trial), int(dim), int(s), int(i))


def lattice(dim, divisions, level, uid, split=2):
    K = (C.c_uint64 * MAX_DIM)()
    lo, hi = _split_id(uid)
    lib().oracle_cube_lattice_w(dim, divisions, split, level, lo, hi, K)
    return np.array(K[:dim], dtype=np.uint64)


def bounds(p: Problem, level: int, uid: int):
    lo = (C.c_double * MAX_DIM)()
    h = (C.c_double * MAX_DIM)()
    v = C.c_double()
    a, b = _split_id(uid)
    lib().oracle_cube_bounds_w(C.byref(p), level, a, b, lo, h, C.byref(v))
    return np.array(lo[:p.dim]), np.array(h[:p.dim]), v.value


def f(integrand, params, x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    prm = (C.c_double * MAX_PARAMS)(*[float(v) for v in params])
    return lib().oracle_f(int(integrand), prm, len(x), x.ctypes.data_as(C.POINTER(C.c_double)))


def sample_x(p: Problem, level, uid, trial, s):
    x = (C.c_double * MAX_DIM)()
    a, b = _split_id(uid)
    lib().oracle_sample_x_w(C.byref(p), level, a, b, trial, int(s), x)
    return np.array(x[:p.dim])


def cube_trial(p: Problem, level, uid, trial):
    I, S1, S2, SA = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    a, b = _split_id(uid)
    st = lib().oracle_cube_trial_w(C.byref(p), level, a, b, trial, C.byref(I), C.byref(S1), C.byref(S2),
                                   C.byref(SA))
    return st, I.value, S1.value, S2.value, SA.value


def cube(p: Problem, level, uid):
    I = (C.c_double * p.trials)()
    m, s, sa = C.c_double(), C.c_double(), C.c_double()
    a, b = _split_id(uid)
    st = lib().oracle_cube_w(C.byref(p), level, a, b, I, C.byref(m), C.byref(s), C.byref(sa))
    return st, np.array(I[:]), m.value, s.value, sa.value


def threshold(s, sigma_mult):
    s = np.ascontiguousarray(s, dtype=np.float64)
    mu, sd = C.c_double(), C.c_double()
    thr = lib().oracle_threshold(s.ctypes.data_as(C.POINTER(C.c_double)), len(s), float(sigma_mult),
                                 C.byref(mu), C.byref(sd))
    return thr, mu.value, sd.value


def children(uid, dim, split=2):
    """The children's ids bits 0..63 (np.uint64); see children_w."""
    return children_w(uid, dim, split)[0]


def children_w(uid, dim, split=2):
    """The children's ids as (bits 0..63 as np.uint64, bits 64..83 as
    np.uint32)."""
    out = (C.c_uint64 * (split ** dim))()
    out_hi = (C.c_uint32 * (split ** dim))()
    a, b = _split_id(uid)
    lib().oracle_children_w(a, b, dim, split, out, out_hi)
    return np.array(out[:], dtype=np.uint64), np.array(out_hi[:], dtype=np.uint32)


def validate(p: Problem) -> int:
    return lib().oracle_validate(C.byref(p))


@dataclass
class Level:
    n: int
    uid: np.ndarray      # id bits 0..63
    uid_hi: np.ndarray   # id bits 64..83
    m: np.ndarray
    s: np.ndarray
    I: np.ndarray
    sa: np.ndarray
    sel: np.ndarray
    thr: float
    mu: float
    sd: float
    min_margin: float
    n_sel: int
    n_in_band: int
    n_replayed: int


@dataclass
class Run:
    status: int
    flags: int
    integral: float = float("nan")
    std: float = float("nan")
    stderr: float = float("nan")
    sum_abs: float = float("nan")
    n_samples: int = 0
    n_cubes: int = 0
    levels: list = field(default_factory=list)


def integrate(p: Problem, replay=None, band_eps: float = 0.0) -> Run:
    """Run the whole tree search.  ``replay``: list (per level) of (uids, sel)
    or (uids, sel, uids_hi) from another run; decisions inside the
    ``band_eps`` margin are adopted."""
    L = lib()
    rp = None
    keep = []
    if replay is not None:
        rp = Replay()
        rp.n_levels = len(replay)
        for l, item in enumerate(replay):
            u, s = item[0], item[1]
            uh = item[2] if len(item) > 2 and item[2] is not None else np.zeros(len(u), np.uint32)
            u = np.ascontiguousarray(u, dtype=np.uint64)
            s = np.ascontiguousarray(s, dtype=np.uint8)
            uh = np.ascontiguousarray(uh, dtype=np.uint32)
            order = np.lexsort((u, uh))  # by (uid_hi, uid)
            u, s, uh = (np.ascontiguousarray(u[order]), np.ascontiguousarray(s[order]),
                        np.ascontiguousarray(uh[order]))
            keep += [u, s, uh]
            rp.n[l] = len(u)
            rp.uid[l] = u.ctypes.data_as(C.POINTER(C.c_uint64))
            rp.uid_hi[l] = uh.ctypes.data_as(C.POINTER(C.c_uint32))
            rp.sel[l] = s.ctypes.data_as(C.POINTER(C.c_uint8))
    h = L.oracle_integrate(C.byref(p), C.byref(rp) if rp is not None else None, float(band_eps))
    if not h:
        raise MemoryError("oracle_integrate")
    try:
        run = Run(status=L.oracle_run_status(h), flags=L.oracle_run_flags(h))
        tot = (C.c_double * 4)()
        cnt = (C.c_uint64 * 2)()
        L.oracle_run_totals(h, tot, cnt)
        run.integral, run.std, run.stderr, run.sum_abs = tot[0], tot[1], tot[2], tot[3]
        run.n_samples, run.n_cubes = int(cnt[0]), int(cnt[1])
        for l in range(L.oracle_run_levels(h)):
            n = int(L.oracle_level_n(h, l))
            st = (C.c_double * 4)()
            cc = (C.c_int64 * 3)()
            L.oracle_level_stats(h, l, st, cc)

            def arr(fn, count, dt):
                ptr = fn(h, l)
                if count == 0 or not ptr:
                    return np.zeros(0, dtype=dt)
                return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dt, copy=True)

            run.levels.append(Level(
                n=n,
                uid=arr(L.oracle_level_uid, n, np.uint64),
                uid_hi=arr(L.oracle_level_uid_hi, n, np.uint32),
                m=arr(L.oracle_level_m, n, np.float64),
                s=arr(L.oracle_level_s, n, np.float64),
                I=arr(L.oracle_level_I, n * p.trials, np.float64).reshape(n, p.trials),
                sa=arr(L.oracle_level_sa, n, np.float64),
                sel=arr(L.oracle_level_sel, n, np.uint8),
                thr=st[0], mu=st[1], sd=st[2], min_margin=st[3],
                n_sel=int(cc[0]), n_in_band=int(cc[1]), n_replayed=int(cc[2])))
        return run
    finally:
        L.oracle_free(h)
