"""ctypes mirror of ``include/zmc.h`` and the loader of ``libzmc.so``.

Argument marshalling only: every step of the integration runs in the HIP
library.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libzmc.so")

MAX_DIM = 16
MAX_LEVELS = 16
MAX_PARAMS = 2 * MAX_DIM + 2

# zmc_status
OK, EINVAL, ENOMEM, ENONFINITE, EDEVICE, EAGAIN, EBUSY, ENOINIT, ECANCELED, ENOTFOUND = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9)
# zmc_integrand
GAUSS, SIN_SUM, GENZ_OSC, GENZ_PPEAK, GENZ_CPEAK, GENZ_GAUSS, CONST, MONOMIAL = range(8)
INTEGRANDS = {"gauss": GAUSS, "sin_sum": SIN_SUM, "genz_osc": GENZ_OSC, "genz_ppeak": GENZ_PPEAK,
              "genz_cpeak": GENZ_CPEAK, "genz_gauss": GENZ_GAUSS, "const": CONST, "monomial": MONOMIAL}
# zmc_eval
EVAL_FP64, EVAL_FP32 = 0, 1
F_TRUNCATED, F_RTOL_MET, F_FP32_RANGE = 1, 2, 4

EXPORTS = ("zmc_init", "zmc_shutdown", "zmc_integrate", "zmc_integrate_request", "zmc_integrate_batch",
           "zmc_submit", "zmc_poll", "zmc_cancel", "zmc_serve_stats", "zmc_debug_philox", "zmc_debug_points",
           "zmc_cube_estimates", "zmc_strerror", "zmc_version", "zmc_struct_size", "zmc_register_integrand",
           "zmc_request_bytes", "zmc_integrate_noalloc")


class Result(C.Structure):
    _fields_ = [
        ("integral", C.c_double), ("std", C.c_double), ("stderr_", C.c_double),
        ("n_samples", C.c_uint64), ("n_cubes", C.c_uint64),
        ("levels_run", C.c_int32), ("flags", C.c_int32), ("status", C.c_int32), ("reserved", C.c_int32),
        ("cubes_per_level", C.c_uint64 * MAX_LEVELS), ("selected_per_level", C.c_uint64 * MAX_LEVELS),
        ("thr_per_level", C.c_double * MAX_LEVELS), ("min_margin_per_level", C.c_double * MAX_LEVELS),
        ("ms_per_level", C.c_float * MAX_LEVELS), ("sample_ms_per_level", C.c_float * MAX_LEVELS),
        ("sample_launches_per_level", C.c_int32 * MAX_LEVELS), ("latency_ms", C.c_double),
    ]


class Request(C.Structure):
    _fields_ = [
        ("integrand", C.c_int32), ("dim", C.c_int32), ("divisions_per_axis", C.c_int32),
        ("trials", C.c_int32), ("max_depth", C.c_int32), ("eval", C.c_int32), ("n_params", C.c_int32),
        ("split", C.c_int32), ("threshold_scope", C.c_int32),
        ("reserved", C.c_int32), ("samples_per_cube", C.c_int64), ("max_cubes_per_level", C.c_int64),
        ("sigma_mult", C.c_double), ("rtol", C.c_double), ("seed", C.c_uint64),
        ("lower", C.c_double * MAX_DIM), ("upper", C.c_double * MAX_DIM), ("params", C.c_double * MAX_PARAMS),
    ]


class Config(C.Structure):
    _fields_ = [
        ("arena", C.c_void_p), ("arena_bytes", C.c_uint64), ("max_slots", C.c_int32),
        ("queue_depth", C.c_int32), ("serve_stream", C.c_void_p), ("tune_path", C.c_char_p),
        ("serve_lanes", C.c_int32), ("default_eval", C.c_int32), ("serve_chunk_samples", C.c_int64),
    ]


class Trace(C.Structure):
    _fields_ = [
        ("max_levels", C.c_int32), ("reserved", C.c_int32), ("capacity", C.c_int64),
        ("n", C.c_int64 * MAX_LEVELS),
        ("uid", C.POINTER(C.c_uint64) * MAX_LEVELS), ("m", C.POINTER(C.c_double) * MAX_LEVELS),
        ("s", C.POINTER(C.c_double) * MAX_LEVELS), ("sel", C.POINTER(C.c_uint8) * MAX_LEVELS),
        ("S1", C.POINTER(C.c_double) * MAX_LEVELS), ("S2", C.POINTER(C.c_double) * MAX_LEVELS),
        ("uid_hi", C.POINTER(C.c_uint32) * MAX_LEVELS),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Load libzmc.so and declare its signatures.  Raises if it is missing:
    there is no fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libzmc.so is not built (%s); run `python -m paper_1902_07916_amd.build`" % path)
    L = C.CDLL(path)
    vp, i32, i64, u32, u64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
    R, Q = C.POINTER(Result), C.POINTER(Request)
    L.zmc_init.argtypes = [C.POINTER(Config)]
    L.zmc_shutdown.argtypes = []
    L.zmc_integrate.argtypes = [i32, C.POINTER(dbl), i32, C.POINTER(dbl), C.POINTER(dbl), i32, i64, i32, i32, dbl,
                                u64, vp, R]
    L.zmc_integrate_request.argtypes = [Q, vp, R, C.POINTER(Trace)]
    L.zmc_integrate_batch.argtypes = [Q, i32, vp, R]
    L.zmc_submit.argtypes = [Q, C.POINTER(u64)]
    L.zmc_poll.argtypes = [u64, R, i32]
    L.zmc_cancel.argtypes = [u64]
    L.zmc_serve_stats.argtypes = [C.POINTER(u64)]
    L.zmc_debug_philox.argtypes = [u32, u32, C.POINTER(u32), i64, C.POINTER(u32), vp]
    L.zmc_debug_points.argtypes = [Q, i32, u64, i32, i64, i64, C.POINTER(dbl), vp]
    L.zmc_cube_estimates.argtypes = [Q, i32, C.POINTER(u64), i64, C.POINTER(dbl), C.POINTER(dbl),
                                     C.POINTER(dbl), C.POINTER(dbl), vp]
    L.zmc_strerror.argtypes = [i32]
    L.zmc_strerror.restype = C.c_char_p
    L.zmc_version.argtypes = []
    L.zmc_version.restype = C.c_char_p
    L.zmc_struct_size.argtypes = [i32]
    L.zmc_register_integrand.argtypes = [C.c_char_p, i32, C.POINTER(C.c_int)]
    L.zmc_request_bytes.argtypes = [Q, C.POINTER(u64)]
    L.zmc_integrate_noalloc.argtypes = [Q, vp, R]
    for i, T in enumerate((Result, Request, Config, Trace)):
        if L.zmc_struct_size(i) != C.sizeof(T):
            raise RuntimeError("ABI mismatch for %s: C %d vs ctypes %d" % (T.__name__, L.zmc_struct_size(i),
                                                                          C.sizeof(T)))
    _lib = L
    return L


class ZmcError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = load().zmc_strerror(code).decode(errors="replace")
        super().__init__("%s failed: %d (%s)" % (where, code, msg))


def check(code: int, where: str) -> int:
    if code != OK:
        raise ZmcError(code, where)
    return code
