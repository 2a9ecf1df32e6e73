"""MI355X (gfx950) stratified-sampling + heuristic tree-search Monte Carlo
integrator -- the method of ZMCintegral (arXiv:1902.07916, Sec. 2).

Thin Python binding of ``libzmc.so`` (declared in ``include/zmc.h``): PyTorch
provides the device arena and the streams; every step of the integration runs
in the library's HIP kernels.  There is no CPU fallback: constructing an
:class:`Integrator` without the built library, or without a GPU, raises.

    from paper_1902_07916_amd import Integrator
    zi = Integrator(arena_bytes=4 << 30)
    r = zi.integrate("sin_sum", [], [0.0] * 6, [10.0] * 6, divisions=6,
                     samples=16384, trials=5, max_depth=2, sigma_mult=1.0,
                     seed=1, eval="fp32")
    print(r.integral, r.stderr)
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np

from . import _abi
from ._abi import (CONST, EVAL_FP32, EVAL_FP64, F_FP32_RANGE, F_RTOL_MET, F_TRUNCATED, GAUSS, GENZ_CPEAK, GENZ_GAUSS,
                   GENZ_OSC, GENZ_PPEAK, INTEGRANDS, MONOMIAL, SIN_SUM, ZmcError, check)

__all__ = ["Integrator", "Result", "make_request", "register_integrand", "ZmcError", "INTEGRANDS", "GAUSS", "SIN_SUM", "GENZ_OSC",
           "GENZ_PPEAK", "GENZ_CPEAK", "GENZ_GAUSS", "CONST", "MONOMIAL", "EVAL_FP64", "EVAL_FP32",
           "F_TRUNCATED", "F_RTOL_MET", "F_FP32_RANGE"]


def _integrand_id(x) -> int:
    if isinstance(x, str):
        return INTEGRANDS[x]
    return int(x)


def _eval_id(x) -> int:
    if isinstance(x, str):
        return {"fp64": EVAL_FP64, "fp32": EVAL_FP32}[x]
    return int(x)


def make_request(integrand, params, lower, upper, divisions, samples, trials, max_depth, sigma_mult, seed,
                 eval="fp64", rtol=0.0, max_cubes_per_level=0, split=0, threshold_scope=0) -> _abi.Request:
    """Fill a zmc_request; lower/upper may be scalars (broadcast to dim).
    split: parts per axis of a split (0/2 = bisection); threshold_scope: 0 per
    level, 1 per parent."""
    params = [float(v) for v in params]
    lower = np.atleast_1d(np.asarray(lower, dtype=np.float64))
    upper = np.atleast_1d(np.asarray(upper, dtype=np.float64))
    dim = max(len(lower), len(upper))
    lower = np.broadcast_to(lower, (dim,))
    upper = np.broadcast_to(upper, (dim,))
    r = _abi.Request()
    r.integrand = _integrand_id(integrand)
    r.dim = dim
    r.divisions_per_axis = int(divisions)
    r.trials = int(trials)
    r.max_depth = int(max_depth)
    r.eval = _eval_id(eval)
    r.n_params = len(params)
    r.samples_per_cube = int(samples)
    r.max_cubes_per_level = int(max_cubes_per_level)
    r.split = int(split)
    r.threshold_scope = int(threshold_scope)
    r.sigma_mult = float(sigma_mult)
    r.rtol = float(rtol)
    r.seed = int(seed) & ((1 << 64) - 1)
    if dim > _abi.MAX_DIM or len(params) > _abi.MAX_PARAMS:
        r.dim = dim if dim <= 1 << 20 else 1 << 20
        r.n_params = len(params)
        return r  # the library rejects it with EINVAL
    for i in range(dim):
        r.lower[i] = float(lower[i])
        r.upper[i] = float(upper[i])
    for j, v in enumerate(params):
        r.params[j] = v
    return r


def register_integrand(body: str, n_params: int = 0) -> int:
    """Compile a user integrand (see zmc_register_integrand in zmc.h) and
    return its id, usable wherever an integrand id or name is accepted.
    Raises ZmcError (EINVAL, with the compiler log) if it does not compile."""
    L = _abi.load()
    out = C.c_int()
    check(L.zmc_register_integrand(body.encode(), int(n_params), C.byref(out)), "zmc_register_integrand")
    return out.value


def request_from_dict(d: dict) -> _abi.Request:
    keys = ("integrand", "params", "lower", "upper", "divisions", "samples", "trials", "max_depth",
            "sigma_mult", "seed")
    kw = {k: d[k] for k in keys}
    return make_request(**kw, eval=d.get("eval", "fp64"), rtol=d.get("rtol", 0.0),
                        max_cubes_per_level=d.get("max_cubes_per_level", 0), split=d.get("split", 0),
                        threshold_scope=d.get("scope", 0))


@dataclass
class Result:
    integral: float
    std: float
    stderr: float
    n_samples: int
    n_cubes: int
    levels_run: int
    flags: int
    status: int
    cubes_per_level: list
    selected_per_level: list
    thr_per_level: list
    min_margin_per_level: list
    ms_per_level: list
    sample_ms_per_level: list
    sample_launches_per_level: list
    latency_ms: float
    trace: dict = field(default=None, repr=False)

    @classmethod
    def from_c(cls, r: _abi.Result, trace=None) -> "Result":
        L = r.levels_run
        return cls(r.integral, r.std, r.stderr_, int(r.n_samples), int(r.n_cubes), L, r.flags, r.status,
                   [int(v) for v in r.cubes_per_level[:L]], [int(v) for v in r.selected_per_level[:L]],
                   list(r.thr_per_level[:L]), list(r.min_margin_per_level[:L]), list(r.ms_per_level[:L]),
                   list(r.sample_ms_per_level[:L]), list(r.sample_launches_per_level[:L]), r.latency_ms, trace)


class Integrator:
    """Owns the device arena (a torch uint8 tensor) and the library context.

    arena_bytes: device memory for all levels of the trees; serve: start
    serving (the arena is split 1/4 synchronous, 3/4 serving); serve_lanes:
    serving lanes, each an engine with its own thread, stream and equal share
    of the serving arena (0 = the library's default of 2);
    serve_chunk_samples: samples per sampling launch in serving (0 = the
    library's default, -1 = one launch per level); default_eval: the
    evaluation mode of the scalar zmc_integrate entry point.  The library holds
    one context per process: opening an Integrator closes the one open before
    it, whose calls then raise."""

    _active = None

    def __init__(self, arena_bytes: int = 4 << 30, serve: bool = False, max_slots: int = 0, queue_depth: int = 0,
                 tune_path: str | None = None, device: int = 0, serve_lanes: int = 0,
                 serve_chunk_samples: int = 0, default_eval="fp64"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Integrator needs a ROCm GPU (torch.cuda.is_available() is False)")
        self._lib = _abi.load()
        torch.cuda.set_device(device)
        self.device = device
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
        self.serve_stream = torch.cuda.Stream() if serve else None
        cfg = _abi.Config()
        cfg.arena = self.arena.data_ptr()
        cfg.arena_bytes = int(arena_bytes)
        cfg.max_slots = int(max_slots)
        cfg.queue_depth = int(queue_depth)
        cfg.serve_stream = self.serve_stream.cuda_stream if serve else None
        cfg.serve_lanes = int(serve_lanes)
        cfg.serve_chunk_samples = int(serve_chunk_samples)
        cfg.default_eval = _eval_id(default_eval)
        self._tune = tune_path.encode() if tune_path else None
        cfg.tune_path = self._tune
        if Integrator._active is not None and Integrator._active is not self:
            Integrator._active.close()
        check(self._lib.zmc_init(C.byref(cfg)), "zmc_init")
        Integrator._active = self
        self._open = True

    # -- lifecycle -------------------------------------------------------------
    def close(self):
        if getattr(self, "_open", False):
            self._lib.zmc_shutdown()
            self._open = False
            if Integrator._active is self:
                Integrator._active = None
            self.arena = None
            self.serve_stream = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _live(self):
        if not getattr(self, "_open", False):
            raise RuntimeError("this Integrator is closed (the library holds one context per process, and opening "
                               "another Integrator closes the previous one)")
        return self._lib

    @staticmethod
    def _stream():
        import torch
        return torch.cuda.current_stream().cuda_stream

    # -- synchronous integration ----------------------------------------------
    def integrate(self, integrand, params, lower, upper, divisions, samples, trials, max_depth, sigma_mult, seed,
                  eval="fp64", rtol=0.0, max_cubes_per_level=0, split=0, scope=0, trace: bool = False,
                  trace_capacity: int = 1 << 20, raise_on_error: bool = True) -> Result:
        req = make_request(integrand, params, lower, upper, divisions, samples, trials, max_depth, sigma_mult,
                           seed, eval, rtol, max_cubes_per_level, split, scope)
        return self.integrate_request(req, trace=trace, trace_capacity=trace_capacity,
                                      raise_on_error=raise_on_error)

    def integrate_request(self, req: _abi.Request, trace: bool = False, trace_capacity: int = 1 << 20,
                          raise_on_error: bool = True) -> Result:
        self._live()
        out = _abi.Result()
        tr = None
        bufs = None
        if trace:
            tr, bufs = self._make_trace(req, trace_capacity)
        rc = self._lib.zmc_integrate_request(C.byref(req), self._stream(), C.byref(out),
                                             C.byref(tr) if tr is not None else None)
        if rc != 0 and raise_on_error:
            raise ZmcError(rc, "zmc_integrate_request")
        tdict = None
        if trace:
            tdict = self._collect_trace(tr, bufs, req, out.levels_run)
        return Result.from_c(out, tdict)

    def integrate_noalloc(self, req: _abi.Request, raise_on_error: bool = True) -> Result:
        """zmc_integrate_noalloc: the request on the library's static device
        scratch (64 MiB), allocating nothing during the call."""
        self._live()
        out = _abi.Result()
        rc = self._lib.zmc_integrate_noalloc(C.byref(req), self._stream(), C.byref(out))
        if rc != 0 and raise_on_error:
            raise ZmcError(rc, "zmc_integrate_noalloc")
        return Result.from_c(out)

    def request_bytes(self, req: _abi.Request) -> int:
        """zmc_request_bytes: worst-case device bytes of the request's tree."""
        out = C.c_uint64()
        check(self._lib.zmc_request_bytes(C.byref(req), C.byref(out)), "zmc_request_bytes")
        return out.value

    def integrate_batch(self, reqs) -> list:
        self._live()
        arr = (_abi.Request * len(reqs))(*reqs)
        outs = (_abi.Result * len(reqs))()
        rc = self._lib.zmc_integrate_batch(arr, len(reqs), self._stream(), outs)
        if rc not in (0, _abi.ENOMEM, _abi.ENONFINITE):
            raise ZmcError(rc, "zmc_integrate_batch")
        return [Result.from_c(o) for o in outs]

    # -- serving ---------------------------------------------------------------
    def submit(self, req: _abi.Request) -> int:
        self._live()
        t = C.c_uint64()
        check(self._lib.zmc_submit(C.byref(req), C.byref(t)), "zmc_submit")
        return t.value

    def poll(self, ticket: int, wait: bool = False):
        self._live()
        out = _abi.Result()
        rc = self._lib.zmc_poll(ticket, C.byref(out), 1 if wait else 0)
        if rc == _abi.EAGAIN:
            return None
        check(rc, "zmc_poll")
        return Result.from_c(out)

    def cancel(self, ticket: int):
        self._live()
        check(self._lib.zmc_cancel(ticket), "zmc_cancel")

    def serve_stats(self):
        self._live()
        out = (C.c_uint64 * 4)()
        check(self._lib.zmc_serve_stats(out), "zmc_serve_stats")
        return dict(queued=out[0], resident=out[1], completed=out[2], levels=out[3])

    # -- step-level access for parity checks -----------------------------------
    def debug_philox(self, key, ctr: np.ndarray) -> np.ndarray:
        self._live()
        ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
        out = np.zeros_like(ctr)
        check(self._lib.zmc_debug_philox(int(key[0]), int(key[1]), ctr.ctypes.data_as(C.POINTER(C.c_uint32)),
                                         len(ctr), out.ctypes.data_as(C.POINTER(C.c_uint32)), self._stream()),
              "zmc_debug_philox")
        return out

    def debug_points(self, req: _abi.Request, level: int, uid: int, trial: int, s0: int, n: int) -> np.ndarray:
        self._live()
        x = np.zeros((n, req.dim), dtype=np.float64)
        check(self._lib.zmc_debug_points(C.byref(req), level, int(uid), trial, s0, n,
                                         x.ctypes.data_as(C.POINTER(C.c_double)), self._stream()),
              "zmc_debug_points")
        return x

    def cube_estimates(self, req: _abi.Request, level: int, uids, sums: bool = True):
        self._live()
        uids = np.ascontiguousarray(uids, dtype=np.uint64)
        n = len(uids)
        m = np.zeros(n)
        s = np.zeros(n)
        S1 = np.zeros((n, req.trials)) if sums else None
        S2 = np.zeros((n, req.trials)) if sums else None
        P = C.POINTER(C.c_double)
        check(self._lib.zmc_cube_estimates(C.byref(req), level, uids.ctypes.data_as(C.POINTER(C.c_uint64)), n,
                                           m.ctypes.data_as(P), s.ctypes.data_as(P),
                                           S1.ctypes.data_as(P) if sums else None,
                                           S2.ctypes.data_as(P) if sums else None, self._stream()),
              "zmc_cube_estimates")
        return m, s, S1, S2

    # -- trace helpers ---------------------------------------------------------
    def _make_trace(self, req, capacity):
        tr = _abi.Trace()
        tr.max_levels = _abi.MAX_LEVELS
        tr.capacity = capacity
        bufs = []
        for l in range(min(req.max_depth + 1, _abi.MAX_LEVELS)):
            b = dict(uid=np.zeros(capacity, np.uint64), uid_hi=np.zeros(capacity, np.uint32), m=np.zeros(capacity),
                     s=np.zeros(capacity), sel=np.zeros(capacity, np.uint8), S1=np.zeros(capacity * req.trials),
                     S2=np.zeros(capacity * req.trials))
            tr.uid[l] = b["uid"].ctypes.data_as(C.POINTER(C.c_uint64))
            tr.uid_hi[l] = b["uid_hi"].ctypes.data_as(C.POINTER(C.c_uint32))
            tr.m[l] = b["m"].ctypes.data_as(C.POINTER(C.c_double))
            tr.s[l] = b["s"].ctypes.data_as(C.POINTER(C.c_double))
            tr.sel[l] = b["sel"].ctypes.data_as(C.POINTER(C.c_uint8))
            tr.S1[l] = b["S1"].ctypes.data_as(C.POINTER(C.c_double))
            tr.S2[l] = b["S2"].ctypes.data_as(C.POINTER(C.c_double))
            bufs.append(b)
        return tr, bufs

    @staticmethod
    def _collect_trace(tr, bufs, req, levels):
        out = []
        for l in range(min(levels, len(bufs))):
            n = int(tr.n[l])
            c = min(n, len(bufs[l]["uid"]))
            b = bufs[l]
            out.append(dict(n=n, uid=b["uid"][:c].copy(), uid_hi=b["uid_hi"][:c].copy(), m=b["m"][:c].copy(),
                            s=b["s"][:c].copy(),
                            sel=b["sel"][:c].copy(), S1=b["S1"][:c * req.trials].reshape(c, req.trials).copy(),
                            S2=b["S2"][:c * req.trials].reshape(c, req.trials).copy()))
        return out

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
