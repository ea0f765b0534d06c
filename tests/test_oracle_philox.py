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


def _chi2_p(counts):
    from scipy.stats import chi2
    counts = np.asarray(counts, dtype=np.float64).ravel()
    exp = counts.sum() / counts.size
    return chi2.sf(((counts - exp) ** 2 / exp).sum(), counts.size - 1)


def test_philox_streams_horizontal_and_vertical(orc):
    """A small battery in the spirit of appendix A.4, on the streams the
    kernels actually draw: across sites at one sweep (the horizontal
    order, one draw per thread), across heat-bath sweeps at one site, across
    replicas and across samples.  For each: every byte of every word is
    flat, pairs of consecutive 23-bit uniforms are flat on a 16 x 16 grid,
    and consecutive uniforms are uncorrelated."""
    n = 1 << 14
    key = [0x13091599, 0x2013]
    streams = {
        "sites": [[i, 5, 0, orc.ctr3(0, 3, 1)] for i in range(n)],
        "sweeps": [[77, s, 0, orc.ctr3(0, 3, 1)] for s in range(n)],
        "replicas x slots": [[77, 5, 0, orc.ctr3(0, k, r)] for r in range(64) for k in range(n // 64)],
        "samples": [[77, 5, m, orc.ctr3(0, 3, 1)] for m in range(n)],
    }
    for name, ctrs in streams.items():
        w = np.array([orc.philox(key, c) for c in ctrs], dtype=np.uint32)        # (n, 4)
        for j in range(4):
            for b in range(4):
                byte = (w[:, j] >> np.uint32(8 * b)) & np.uint32(0xFF)
                assert _chi2_p(np.bincount(byte, minlength=256)) > 1e-4, (name, j, b)
        u = (w[:, 0] >> np.uint32(9)).astype(np.float64) / 2 ** 23
        pairs = np.histogram2d(u[:-1], u[1:], bins=16, range=[[0, 1], [0, 1]])[0]
        assert _chi2_p(pairs) > 1e-4, name
        r = np.corrcoef(u[:-1], u[1:])[0, 1]
        assert abs(r) < 4 / np.sqrt(n), (name, r)
        # the two words one heat-bath update uses are independent of each other
        u1 = (w[:, 1] >> np.uint32(9)).astype(np.float64) / 2 ** 23
        assert abs(np.corrcoef(u, u1)[0, 1]) < 4 / np.sqrt(n), name
        assert _chi2_p(np.histogram2d(u, u1, bins=16, range=[[0, 1], [0, 1]])[0]) > 1e-4, name
