"""Pins of the oracle's Philox4x32-10 and of its uniform mapping.

Philox is pinned to the published known-answer vectors (tests/golden) and, word
for word, to rocRAND's independent host-side implementation.  The uniform
mapping is pinned to its exact special cases and to a Kolmogorov-Smirnov test.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_known_answer_vectors(orc):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert list(orc.philox(ctr, key)) == out


@pytest.fixture(scope="module")
def rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available for the rocRAND host reference")
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    exe = os.path.join(out_dir, "philox_rocrand")
    src = os.path.join(HERE, "philox_rocrand.cpp")
    if not os.path.exists(exe) or os.path.getmtime(exe) < os.path.getmtime(src):
        subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-o", exe, src],
                       check=True, capture_output=True)
    return exe


def test_matches_rocrand_word_for_word(orc, rocrand_ref):
    rng = np.random.default_rng(2024)
    cases = rng.integers(0, 2**32, size=(2000, 6), dtype=np.uint64)
    # include structured counters of the shape the integrator uses
    cases[:8] = [[0, 0, 0, 0, 1, 0], [1, 0, 0, 0, 1, 0], [0, 1, 0, 0, 1, 0], [0, 0, 1, 0, 1, 0],
                 [0, 0, 0, 1, 1, 0], [5, 4 | (3 << 8), 123, 0, 7, 0], [2**32 - 1, 255, 2**32 - 1, 2**32 - 1,
                                                                      2**32 - 1, 2**32 - 1], [0, 0, 0, 0, 0, 0]]
    text = "\n".join(" ".join("%08x" % int(v) for v in row) for row in cases) + "\n"
    res = subprocess.run([rocrand_ref], input=text, capture_output=True, text=True, check=True)
    ref = [[int(t, 16) for t in line.split()] for line in res.stdout.strip().splitlines()]
    assert len(ref) == len(cases)
    for row, r in zip(cases, ref):
        assert list(orc.philox(row[:4], row[4:6])) == r


def test_word_layout_selects_lane(orc):
    # word n of the (seed, uid, level, trial) stream is lane n&3 of block n>>2
    seed, uid, level, trial, D = 0x0123456789ABCDEF, (7 << 32) | 99, 3, 4, 5
    key = (seed & 0xFFFFFFFF, seed >> 32)
    for s in range(0, 9):
        for i in range(D):
            n = s * D + i
            blk = orc.philox((n >> 2, trial | (level << 8), uid & 0xFFFFFFFF, uid >> 32), key)
            assert orc.word(seed, uid, level, trial, D, s, i) == blk[n & 3]


def test_uniform_special_cases(orc):
    assert orc.uniform(0) == 2.0**-24
    assert orc.uniform(0x1FF) == 2.0**-24              # low 9 bits are ignored
    assert orc.uniform(0x200) == 3 * 2.0**-24
    assert orc.uniform(0xFFFFFFFF) == 1.0 - 2.0**-24
    assert orc.uniform(0x80000000) == 0.5 + 2.0**-24
    # every value is an odd multiple of 2^-24 strictly inside (0, 1) and exact in FP32
    for w in np.random.default_rng(1).integers(0, 2**32, 5000):
        u = orc.uniform(int(w))
        assert 0.0 < u < 1.0
        k = u * 2**24
        assert k == int(k) and int(k) % 2 == 1
        assert float(np.float32(u)) == u


def test_uniform_stream_is_uniform(orc):
    # Kolmogorov-Smirnov on the words that drive one cube's samples
    p = orc.problem(orc.SIN_SUM, 3, 0.0, 1.0, 2, 6000, 2, 0, 1.0, 42)
    us = []
    for s in range(6000):
        x = orc.sample_x(p, 0, 5, 1, s)
        lo, h, _ = orc.bounds(p, 0, 5)
        us.extend(((x - lo) / h).tolist())
    us = np.array(us)
    assert us.min() > 0 and us.max() < 1
    assert stats.kstest(us, "uniform").pvalue > 1e-4
    # consecutive dims are uncorrelated
    u3 = us.reshape(-1, 3)
    assert abs(np.corrcoef(u3[:, 0], u3[:, 1])[0, 1]) < 0.05
