"""CPU checks of bench.py's host logic: the one-GPU guard, the reading of
the committed rocprofv3 --pmc summary behind the traffic field, and the
oracle CPU baseline on small lattices, single-L and mixed-L."""
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_1309_1599_amd import inputs  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=60)
    assert out.returncode == 2 and "one GPU" in out.stderr and out.stdout == ""


@pytest.mark.parametrize("preset", ["L64x8", "L32x64", "L64x8_bimodal"])
def test_pmc_summary_is_read_only_for_its_kernel_and_mapping(preset):
    text = open(bench.PMC_SUMMARY.format(preset=preset)).read()
    h = re.search(r"kernel_source_sha256:\s*([0-9a-f]{16})", text).group(1)
    mapping = re.search(r"mapping:\s*(\w+)", text).group(1)
    b = bench.pmc_traffic(preset, mapping, h)
    assert b is not None and b > 0
    # per launch: bytes per update x updates per launch, as the summary states
    upd = float(re.search(r"updates per launch:\s*([0-9]+)", text).group(1))
    per = float(re.search(r"->\s*([0-9.]+) B per update", text).group(1))
    assert b == pytest.approx(upd * per, rel=1e-3)
    assert bench.pmc_traffic(preset, mapping, "0" * 16) is None
    assert bench.pmc_traffic(preset, "resident", h) is None
    assert bench.pmc_traffic("no_such_preset", mapping, h) is None


def test_cpu_baseline_small_lattice():
    L, seed = 4, 5
    temps = inputs.geometric_temps(0.6, 1.6, 4)
    cpl = inputs.gaussian_couplings(L, seed)
    r = bench.cpu_baseline(L, cpl, temps, seed, 1, L, n_chains=4, n_or=2)
    assert r["kind"] == "oracle" and r["unit"] == "ps/SU" and r["cores"] >= 1
    assert np.isfinite(r["value"]) and r["value"] > 0 and r["single_thread_value"] > 0
    assert f"L={L}" in r["sample"]


def test_mixed_cpu_baseline_weights_each_L_by_its_updates():
    """A mixed batch's figure is the per-L figures weighted by each L's share
    of the step's spin updates (1 HB + L OR per sample)."""
    Ls, R, seed = [4, 4, 6], 2, 7
    temps = [inputs.geometric_temps(0.6, 1.6, T) for T in (3, 3, 2)]
    cpl = [inputs.gaussian_couplings(L, seed, s) for s, L in enumerate(Ls)]
    r = bench.mixed_cpu_baseline(Ls, cpl, temps, R, seed, 1, -1, -1)
    su4 = 2 * (1 + 4) * R * 3 * 4 ** 3
    su6 = (1 + 6) * R * 2 * 6 ** 3
    w4, w6 = su4 / (su4 + su6), su6 / (su4 + su6)
    assert r["per_L"]["4"]["su_share"] == pytest.approx(w4, abs=1e-4)
    assert r["per_L"]["6"]["su_share"] == pytest.approx(w6, abs=1e-4)
    expect = w4 * r["per_L"]["4"]["value"] + w6 * r["per_L"]["6"]["value"]
    assert r["value"] == pytest.approx(expect, rel=1e-3, abs=0.2)
    assert r["kind"] == "oracle" and "L=4" in r["sample"] and "L=6" in r["sample"]
