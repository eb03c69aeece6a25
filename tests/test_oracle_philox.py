"""Pins of the oracle's Philox4x32-10 against an independent implementation.

The oracle writes Philox from its published definition (Salmon et al., SC'11).
rocRAND ships a header-only Philox4x32-10; compiled for the host CPU it gives
an independent implementation to compare with, including counters that carry
across words and keys with high bits set.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    out = tmp_path_factory.mktemp("philox") / "ref"
    src = os.path.join(HERE, "helpers", "philox_rocrand_ref.cpp")
    subprocess.run([hipcc, "-O1", src, "-o", str(out)], check=True, capture_output=True)
    return str(out)


def _run_ref(exe, rows):
    text = "\n".join(" ".join("%x" % v for v in r) for r in rows) + "\n"
    res = subprocess.run([exe], input=text, capture_output=True, text=True, check=True)
    return np.array([[int(x, 16) for x in line.split()] for line in res.stdout.strip().splitlines()],
                    dtype=np.uint64)


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(7)
    rows = []
    # (key_lo, key_hi, c0, c1, c2, c3); c1 < 2^30 keeps rocRAND's offset*4 exact
    rows.append((0, 0, 0, 0, 0, 0))
    rows.append((0xFFFFFFFF, 0xFFFFFFFF, 5, 0, 0xFFFFFFFF, 0xFFFFFFFF))
    rows.append((20260103, 0, 0, 0, 0, 1))
    for _ in range(300):
        k = rng.integers(0, 2 ** 32, size=2)
        c = rng.integers(0, 2 ** 32, size=4)
        c[1] %= 2 ** 30
        rows.append((int(k[0]), int(k[1]), int(c[0]), int(c[1]), int(c[2]), int(c[3])))
    ref = _run_ref(rocrand_ref, rows)
    for r, want in zip(rows, ref):
        got = orc.philox([r[2], r[3], r[4], r[5]], [r[0], r[1]])
        assert [int(x) for x in got] == [int(x) for x in want], r


def test_philox_distinct_streams(orc):
    """Words of different counters/keys differ (a dropped counter word would alias)."""
    base = orc.philox([1, 2, 3, 4], [5, 6])
    for i in range(4):
        c = [1, 2, 3, 4]
        c[i] += 1
        assert not np.array_equal(orc.philox(c, [5, 6]), base)
    for i in range(2):
        k = [5, 6]
        k[i] += 1
        assert not np.array_equal(orc.philox([1, 2, 3, 4], k), base)


def test_u24_uniformity(orc):
    """The uniforms drawn from Philox words are flat on [0, 1)."""
    u = np.array([orc.philox([i, 0, 0, 0], [11, 0])[0] >> 8 for i in range(4000)]) / 2.0 ** 24
    hist, _ = np.histogram(u, bins=10, range=(0, 1))
    chi2 = ((hist - 400.0) ** 2 / 400.0).sum()
    assert chi2 < 30.0  # 9 dof, p ~ 4e-4
