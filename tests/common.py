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
