"""Pins of the oracle's Philox4x32-10 and of its uniform conversions.

The generator is pinned against an independent published implementation:
rocRAND's philox4x32_10 engine, compiled here for the host from its header
(tests/philox_rocrand_ref.cpp) and evaluated at the same (key, counter)
pairs.  The conversions are pinned by their exactness claims.
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
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("rocRAND headers / hipcc not available")
    exe = str(tmp_path_factory.mktemp("philox") / "ref")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-I/opt/rocm/include",
                    os.path.join(HERE, "philox_rocrand_ref.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def _query(exe, rows):
    inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()],
                    dtype=np.uint64)


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(20130906)
    rows = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6]
    rows += [tuple(int(v) for v in rng.integers(0, 2 ** 32, 6, dtype=np.uint64))
             for _ in range(300)]
    # counters of the shapes the simulation uses: (site, sweep, sample, tag|slot|rep)
    for tag in (0, 1, 2):
        for i in (0, 1, 4095, 262143):
            rows.append((12345, 678, i, 17, 3, orc.ctr3(tag, 31, 3)))
    ref = _query(rocrand_ref, rows)
    mine = np.array([orc.philox(r[:2], r[2:]) for r in rows], dtype=np.uint64)
    assert ref.shape == mine.shape
    bad = np.nonzero((ref != mine).any(axis=1))[0]
    assert bad.size == 0, f"first mismatch at row {rows[bad[0]]}: {mine[bad[0]]} vs {ref[bad[0]]}"


def test_uniform23_exact_in_fp32(orc):
    ws = [0, 1, 511, 512, 2 ** 31, 2 ** 32 - 1, 0xDEADBEEF]
    for w in ws:
        u = orc.u23(w)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u
        assert float(np.float32(1.0 - u)) == 1.0 - u
        assert float(np.float32(1.0 - 2.0 * u)) == 1.0 - 2.0 * u
    assert orc.u23(0) == 2.0 ** -24
    assert orc.u23(2 ** 32 - 1) == 1.0 - 2.0 ** -24


def test_uniform52_range_and_exactness(orc):
    assert orc.u52(0, 0) == 2.0 ** -53
    assert orc.u52(2 ** 32 - 1, 2 ** 32 - 1) == 1.0 - 2.0 ** -53
    u = orc.u52(0x12345678, 0x9ABCDEF0)
    m = ((0x12345678 >> 6) << 26) | (0x9ABCDEF0 >> 6)
    assert u == (m + 0.5) / 2.0 ** 52


def test_ctr3_fields(orc):
    assert orc.ctr3(1, 0, 0) == 1 << 28
    assert orc.ctr3(0, 4095, 255) == (4095 << 16) | (255 << 8)
    assert orc.ctr3(2, 5, 3) == (2 << 28) | (5 << 16) | (3 << 8)


def test_philox_uniformity(orc):
    """Sanity: the 23-bit uniforms of consecutive sites are flat (chi-square)."""
    u = np.array([orc.u23(orc.philox([7, 9], [i, 0, 0, 0])[0]) for i in range(20000)])
    hist, _ = np.histogram(u, bins=20, range=(0, 1))
    exp = len(u) / 20
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert chi2 < 45.3  # p ~ 0.001 for 19 dof
