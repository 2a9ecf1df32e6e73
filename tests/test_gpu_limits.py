"""Memory limits through the C ABI: a request whose level does not fit the
arena fails with ZMC_ENOMEM and leaves the library usable; in a batch only
that request fails, and the others give bitwise their results alone."""
import math
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu

ENOMEM = -2


@pytest.fixture(scope="module")
def small_arena():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_07916_amd import Integrator
    z = Integrator(arena_bytes=64 << 20)  # the minimum arena
    yield z
    z.close()


def _huge():
    # 4e6 root cubes of ~100 bytes each: far beyond a 64 MiB arena
    from paper_1902_07916_amd import make_request
    return make_request("gauss", [0.2, 1.0, 0.0, 0.0], [-1.0] * 2, [1.0] * 2, 2000, 64, 5, 0, 1.0, 1)


def _small(seed):
    from paper_1902_07916_amd import make_request
    return make_request("gauss", [0.2, 1.0, 0.0, 0.0], [-1.0] * 2, [1.0] * 2, 8, 512, 5, 2, 1.0, seed)


def test_enomem_then_recovers(small_arena):
    from paper_1902_07916_amd import ZmcError
    print("limits: oversized request", flush=True)
    with pytest.raises(ZmcError) as e:
        small_arena.integrate_request(_huge())
    assert e.value.code == ENOMEM
    r = small_arena.integrate_request(_huge(), raise_on_error=False)
    assert r.status == ENOMEM and math.isnan(r.integral)
    ok = small_arena.integrate_request(_small(1))
    exact = 2 * math.pi * 0.2 ** 2 * math.erf(1 / (0.2 * math.sqrt(2))) ** 2
    assert ok.status == 0 and abs(ok.integral - exact) < 5 * ok.stderr + 1e-12


def test_batch_with_one_oversized(small_arena):
    print("limits: batch with an oversized request", flush=True)
    reqs = [_small(1), _huge(), _small(2)]
    out = small_arena.integrate_batch(reqs)
    assert [r.status for r in out] == [0, ENOMEM, 0]
    for i in (0, 2):
        alone = small_arena.integrate_request(reqs[i])
        assert alone.integral == out[i].integral and alone.std == out[i].std
