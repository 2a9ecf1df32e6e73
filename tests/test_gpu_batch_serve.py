"""Batched and served integration: every integral of a batch (or of the
serving mix) gives bitwise the result it gives alone, and agrees with the
oracle run on that integral alone."""
import os
import sys
import time

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from common import compare_tree, request  # noqa: E402

pytestmark = pytest.mark.gpu

EPS64 = 1e-9
EPS32 = 1e-4


def _small_batch(n, eval_="fp32", seed=7):
    from paper_1902_07916_amd import workloads as W
    # small enough for the oracle: <= 300 root cubes, 128 points, one
    # refinement at sigma 1, next level capped at 20000 cubes (truncation)
    return W.genz_batch(n=n, seed=seed, samples=128, trials=3, max_depth=1, sigma_mult=1.0, eval=eval_,
                        max_root_cubes=300, max_cubes_per_level=20000)


def _same(a, b):
    return (a.integral == b.integral and a.std == b.std and a.cubes_per_level == b.cubes_per_level
            and a.selected_per_level == b.selected_per_level and a.flags == b.flags and a.status == b.status)


@pytest.fixture(scope="module")
def zi():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_07916_amd import Integrator
    z = Integrator(arena_bytes=8 << 30, serve=True)
    yield z
    z.close()


@pytest.mark.parametrize("eval_", ["fp64", "fp32"])
def test_batch_matches_alone_and_oracle(zi, orc, eval_):
    # every member: the batch result is bitwise its result alone, and its
    # traced run alone matches the oracle over the whole tree (decisions
    # inside the rounding band replayed by the oracle)
    ws = _small_batch(24, eval_)
    reqs = [request(w) for w in ws]
    batch = zi.integrate_batch(reqs)
    eps, tol = (EPS64, 1e-6) if eval_ == "fp64" else (EPS32, 1e-4)
    for i, (w, rq, b) in enumerate(zip(ws, reqs, batch)):
        alone = zi.integrate_request(rq)
        assert _same(b, alone), (w, b, alone)
        traced = zi.integrate_request(rq, trace=True)
        assert _same(b, traced)
        print("batch member %d (family %d, D=%d, %d cubes)" % (i, w["integrand"], len(w["lower"]), b.n_cubes),
              flush=True)
        compare_tree(orc, w, traced, eps, tol)


def test_batch_mixed_dims_full_generator(zi):
    # the batched generator's shape: D uniform in 2..12, four families
    from paper_1902_07916_amd import workloads as W
    ws = W.genz_batch(n=64, samples=1024, max_root_cubes=5000)
    reqs = [request(w) for w in ws]
    out = zi.integrate_batch(reqs)
    assert all(r.status == 0 for r in out)
    for i in (0, 17, 63):
        assert _same(out[i], zi.integrate_request(reqs[i]))


def test_serving_mix_matches_alone(zi):
    from paper_1902_07916_amd import workloads as W
    stream = W.serving_stream(rate=400.0, duration=0.1, samples=512, max_root_cubes=2048)
    reqs = [request(w) for _, w in stream]
    assert len(reqs) >= 20
    served = _serve(zi, stream, reqs)
    st = zi.serve_stats()
    assert st["completed"] >= len(reqs) and st["queued"] == 0
    for (_, w), rq, s in zip(stream, reqs, served):
        assert s.status == 0
        alone = zi.integrate_request(rq)
        assert _same(s, alone)
        assert s.latency_ms > 0
    # rtol stop: a met tolerance is a real one
    for rq, s in zip(reqs, served):
        if s.flags & 2:
            assert s.stderr <= (1 + 1e-12) * rq.rtol * abs(s.integral)


def _serve(zi, stream, reqs):
    t0 = time.perf_counter()
    tickets = []
    for (t, w), rq in zip(stream, reqs):
        while time.perf_counter() - t0 < t:
            time.sleep(0.0005)
        tickets.append(zi.submit(rq))
    return [zi.poll(t, wait=True) for t in tickets]


def test_serving_every_request_matches_oracle(zi, orc):
    # a seeded 20-request stream sized for the oracle (the serving mix's
    # roots, 256 points, levels capped at 2^14 cubes): every served result is bitwise
    # its traced run alone, and that run matches the oracle over the whole
    # tree, including the rtol stop
    from paper_1902_07916_amd import workloads as W
    stream = W.serving_stream(rate=400.0, duration=1.0, samples=256,
                              max_cubes_per_level=1 << 14)[:20]
    assert len(stream) == 20
    reqs = [request(w) for _, w in stream]
    served = _serve(zi, stream, reqs)
    for i, ((_, w), rq, s) in enumerate(zip(stream, reqs, served)):
        assert s.status == 0
        traced = zi.integrate_request(rq, trace=True)
        assert _same(s, traced), (i, s, traced)
        print("served request %d (family %d, D=%d, rtol %.2g, levels %s)" % (
            i, w["integrand"], len(w["lower"]), w["rtol"], s.cubes_per_level), flush=True)
        o = compare_tree(orc, w, traced, EPS32, 1e-4)
        assert (o.flags & 2) == (s.flags & 2)


def test_serving_cancel_and_errors(zi):
    from paper_1902_07916_amd import ZmcError, make_request
    # ~2e10 points at the root level: still running when the cancel arrives,
    # unless the submitting thread is descheduled for that long.  One
    # refinement keeps its worst-case tree inside one serving lane's share of
    # the arena (a deeper tree would be refused with ENOMEM at admission).
    big = make_request("genz_osc", [0.1] + [2.0] * 8, [0.0] * 8, [1.0] * 8, 3, 1 << 20, 3, 1, 5.0, 1, eval="fp32")
    t = zi.submit(big)
    zi.cancel(t)
    r = zi.poll(t, wait=True)
    assert r.status in (0, -8)
    with pytest.raises(ZmcError):
        zi.cancel(t)      # collected: unknown now
    # a finished, uncollected request keeps its result when cancelled
    small = make_request("gauss", [0.2, 1.0, 0.0, 0.0], [-1.0] * 2, [1.0] * 2, 4, 256, 3, 1, 1.0, 1)
    t2 = zi.submit(small)
    deadline = time.time() + 30
    while time.time() < deadline:
        st = zi.serve_stats()
        if st["queued"] == 0 and st["resident"] == 0:
            break
        time.sleep(0.001)
    zi.cancel(t2)
    r2 = zi.poll(t2, wait=True)
    assert r2.status == 0 and r2.integral > 0
    with pytest.raises(ZmcError):
        zi.poll(t)        # collected already
    with pytest.raises(ZmcError):
        zi.submit(make_request("gauss", [0.1], [0.0], [1.0], 2, 16, 3, 1, 1.0, 1))  # wrong params


def test_small_level_launch_matches_tiled_path(zi):
    """A level whose segments are all one tile (<= 1024 cubes) runs as one
    launch; the same requests batched with a large one (several tiles) go
    through the per-tile kernels.  Both give bitwise the same results, for
    both threshold scopes and in both precisions."""
    from paper_1902_07916_amd import make_request
    big = make_request("genz_gauss", [2.0] * 4 + [0.3] * 4, [0.0] * 4, [1.0] * 4, 7, 256, 3, 2, 1.0, 5, eval="fp32")
    small = []
    for i, (ev, scope) in enumerate((("fp32", 0), ("fp64", 0), ("fp32", 1), ("fp64", 1))):
        small.append(make_request("gauss", [0.15, 1.0, 0.2, 0.6, 0.4], [0.0] * 3, [1.0] * 3, 5, 300 + 4 * i, 4, 2,
                                  0.5, 11 + i, eval=ev, threshold_scope=scope))
    batch = zi.integrate_batch([big] + small)
    assert batch[0].cubes_per_level[0] == 7 ** 4 > 1024
    for q, b in zip(small, batch[1:]):
        alone = zi.integrate_request(q)
        assert alone.status == 0 and max(alone.cubes_per_level) <= 1024
        assert len(alone.cubes_per_level) == 3 and alone.selected_per_level[0] > 0
        assert _same(b, alone), (b, alone)
