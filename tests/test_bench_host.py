"""CPU checks of bench.py's host logic: the one-GPU guard, the reading of
the committed rocprofv3 --pmc summary behind the traffic field, and the
oracle CPU baseline on a small lattice."""
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


@pytest.mark.parametrize("preset", ["L64x8", "L32x64"])
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
