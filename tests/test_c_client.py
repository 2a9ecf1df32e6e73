"""The library used from plain C through its C ABI alone (tests/c_client.c):
it links against libzmc.so without Python or torch, and on a GPU its
synchronous and served results equal the Python binding's bit for bit and
the oracle's within 1e-6."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CLIENT = os.path.join(HERE, "_build", "c_client")
sys.path.insert(0, HERE)


def test_c_client_links():
    assert os.path.exists(CLIENT), "tests/_build/c_client is built by __graft_entry__.build()"
    out = subprocess.run(["ldd", CLIENT], capture_output=True, text=True, check=True).stdout
    lines = [l for l in out.splitlines() if "libzmc.so" in l]
    assert lines and "not found" not in lines[0], out


@pytest.mark.gpu
def test_c_client_matches_binding_and_oracle(orc):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from common import oracle_problem
    from paper_1902_07916_amd import Integrator
    from paper_1902_07916_amd import workloads as W
    print("c_client: running", flush=True)
    run = subprocess.run([CLIENT], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stderr
    got = {}
    for line in run.stdout.splitlines():
        k, integral, std, levels, samples = line.split()
        got[k] = (float(integral), float(std), int(levels), int(samples))
    w = W.gauss4d(eval="fp64", samples=4096)
    z = Integrator(arena_bytes=256 << 20)
    try:
        r = z.integrate(**w)
    finally:
        z.close()
    o = orc.integrate(oracle_problem(orc, w))
    for k in ("sync", "served"):
        integral, std, levels, samples = got[k]
        assert (integral, std, levels, samples) == (r.integral, r.std, r.levels_run, r.n_samples), k
        assert abs(integral - o.integral) <= 1e-6 * abs(o.integral)
        assert abs(std - o.std) <= 1e-6 * o.std
