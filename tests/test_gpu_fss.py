"""The FSS driver end to end on the GPU at toy sizes: both coupling
families, the chiral channel and the temperature walks are recorded, the
per-bin means are finite and ordered as the physics requires (energy rising
with T, the overlap falling), the report serialises, and a saved batch
loads back unchanged."""
import json

import numpy as np
import pytest

from paper_1309_1599_amd import fss, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"


@pytest.mark.parametrize("couplings", ["bimodal", "gaussian"])
def test_simulate_report_save_load(tmp_path, couplings):
    temps = inputs.geometric_temps(0.9, 1.6, 6)
    S, R, steps, every = 16, 2, 128, 4
    runs = [fss.simulate(L, S, temps, R, steps, every, 77 + L, couplings, 1.0, chiral=True, log=lambda m: None)
            for L in (4, 8)]
    for r in runs:
        assert set(r["means"]) == {"q2", "qk2", "e", "cg2", "cgk2"}
        nb = len(r["bins"])
        assert r["bins"][0] == (steps // every // 2, steps // every)
        assert r["counts"][0] == steps // every // 2
        for v in r["means"].values():
            v = np.asarray(v)
            assert v.shape == (nb, S, len(temps)) and np.isfinite(v).all()
        e = np.asarray(r["means"]["e"])[0].mean(axis=0)
        q2 = np.asarray(r["means"]["q2"])[0].mean(axis=0)
        assert e[-1] > e[0] + 0.1 and np.polyfit(temps, e, 1)[0] > 0, e
        assert q2[0] > q2[-1], q2
        tau = np.asarray(r["tau_walk"])
        assert tau.shape == (S,) and np.isfinite(tau).all()
    res = fss.report(runs, temps, couplings, 1.0)
    json.dumps(res, default=float)
    assert [c["channel"] for c in res["crossings"]] == ["sg", "cg"]
    assert set(res["temperature_walk"]) == {"4", "8"}
    path = tmp_path / "batch.npz"
    fss.save_runs(path, runs)
    back = fss.load_runs([str(path)])
    for a, b in zip(runs, back):
        assert b["n_samples"] == S and b["L"] == a["L"]
        for k in a["means"]:
            np.testing.assert_array_equal(np.asarray(a["means"][k]), b["means"][k])
        np.testing.assert_array_equal(a["tau_walk"], b["tau_walk"])
