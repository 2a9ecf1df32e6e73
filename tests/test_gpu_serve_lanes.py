"""Serving lanes and chunked sampling launches: with several lanes and a
chunk size small enough that every level's sampling is cut into many
launches (the last one ragged), each served integral is bitwise the one the
synchronous path (one launch per bucket and level) gives; the same holds for
a run-time compiled integrand, whose launches take the same unit offsets."""
import os
import sys
import threading
import time

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from common import request  # noqa: E402

pytestmark = pytest.mark.gpu

SIN_BODY = "real t = 0; for (int i = 0; i < D; ++i) t += x[i]; return sin(t);"


def _same(a, b):
    return (a.integral == b.integral and a.std == b.std and a.cubes_per_level == b.cubes_per_level
            and a.selected_per_level == b.selected_per_level and a.flags == b.flags and a.status == b.status)


@pytest.fixture(scope="module")
def zl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_07916_amd import Integrator
    # 3 lanes; 3 * 2^16 + 5 samples per launch: not a multiple of any unit
    z = Integrator(arena_bytes=6 << 30, serve=True, serve_lanes=3, serve_chunk_samples=3 * (1 << 16) + 5)
    yield z
    z.close()


def test_chunked_lanes_match_sync(zl):
    from paper_1902_07916_amd import workloads as W
    stream = W.serving_stream(rate=400.0, duration=0.08, samples=1536, max_root_cubes=2048)
    reqs = [request(w) for _, w in stream]
    assert len(reqs) >= 15
    # submitted in bursts from two threads, so that lanes fill at once
    tickets = [None] * len(reqs)

    def submit(idx):
        for i in idx:
            tickets[i] = zl.submit(reqs[i])

    ths = [threading.Thread(target=submit, args=(range(k, len(reqs), 2),)) for k in range(2)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    served = [zl.poll(t, wait=True) for t in tickets]
    launches = 0
    for rq, s in zip(reqs, served):
        assert s.status == 0
        assert _same(s, zl.integrate_request(rq))
        launches = max(launches, max(s.sample_launches_per_level))
    assert launches > 10  # the levels really were cut into many launches


def test_chunked_ragged_point_counts_match_sync(zl):
    # N not a multiple of 4 takes the masked loop; cut into many launches it
    # must still give bitwise the synchronous result, alone and beside
    # requests of the same bucket with whole groups
    from paper_1902_07916_amd import workloads as W
    base = W.serving_stream(rate=400.0, duration=0.05, samples=1536, max_root_cubes=1024)
    ws = [dict(w, samples=n) for (_, w), n in zip(base[:6], (1537, 1536, 3001, 1538, 4096, 1539))]
    reqs = [request(w) for w in ws]
    tickets = [zl.submit(rq) for rq in reqs]
    served = [zl.poll(t, wait=True) for t in tickets]
    for rq, s in zip(reqs, served):
        assert s.status == 0
        assert _same(s, zl.integrate_request(rq))


def test_chunked_user_integrand_matches_sync(zl):
    import paper_1902_07916_amd as zmc
    from paper_1902_07916_amd import workloads as W
    uid = zmc.register_integrand(SIN_BODY, 0)
    for ev in ("fp32", "fp64"):
        w0 = W.sin6d(eval=ev, samples=2048, divisions=4, max_depth=2)
        rq = request(dict(w0, integrand=uid))
        s = zl.poll(zl.submit(rq), wait=True)
        a = zl.integrate_request(rq)
        assert s.status == 0 and _same(s, a)
        assert max(s.sample_launches_per_level) > 10
        # the built-in kernel, chunked too, gives the same sums in FP64
        b = zl.poll(zl.submit(request(w0)), wait=True)
        assert b.status == 0
        if ev == "fp64":
            assert b.integral == s.integral and b.std == s.std


def test_heavy_lane_leaves_small_requests_to_another(zl):
    # (last in this module: it replaces the module's context with one of
    # default lanes and chunk size)
    # A request whose levels take ~1e11 samples keeps one lane busy; small
    # requests submitted meanwhile are admitted by the other lane, whose
    # launches run between the heavy one's chunks: each finishes in a small
    # fraction of the heavy request's time.
    from paper_1902_07916_amd import Integrator, workloads as W
    zl.close()
    z = Integrator(arena_bytes=12 << 30, serve=True)
    try:
        heavy = request(W.sin6d())
        stream = W.serving_stream(rate=200.0, duration=0.2, samples=512, max_root_cubes=512)
        small = [request(w) for _, w in stream][:8]
        for rq in small:
            z.poll(z.submit(rq), wait=True)
        th = z.submit(heavy)
        time.sleep(0.05)
        res = [z.poll(z.submit(rq), wait=True) for rq in small]
        rh = z.poll(th, wait=True)
        assert rh.status == 0 and all(r.status == 0 for r in res)
        assert max(r.latency_ms for r in res) < 0.1 * rh.latency_ms, ([r.latency_ms for r in res], rh.latency_ms)
    finally:
        z.close()
