"""The FSS driver end to end on the GPU at toy sizes: both coupling
families, the chiral channel and the temperature walks are recorded, the
per-bin means are finite and ordered as the physics requires (energy rising
with T, the overlap falling), the report serialises, and a saved batch
loads back unchanged."""
import json

import numpy as np
import pytest

from paper_1309_1599_amd import analysis as A
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


def _oracle_run(L, cpl, temps, R, steps, every, seed, sample):
    """The FP64 oracle on one sample with fss.simulate's schedule: per
    measurement (after every `every`-th tempering pass) the scalar-overlap
    q(0)^2, |q(k_min)|^2 (mean of the three directions) and the energy per
    spin of each slot; means over the last half of the measurements."""
    import oracle as O
    from oracle import OracleEnsemble
    ens = OracleEnsemble(L, cpl, temps, R, seed, sample=sample)
    T, N = len(temps), L ** 3
    rows = []
    for step in range(1, steps + 1):
        ens.step(1, L)
        ens.swap()
        if step % every == 0:
            q2, qk2, e = np.zeros(T), np.zeros(T), np.zeros(T)
            for k in range(T):
                pairs = [(a, b) for a in range(R) for b in range(a + 1, R)]
                for a, b in pairs:
                    ja, jb = int(ens.perm[a, k]), int(ens.perm[b, k])
                    rec = O.overlaps(L, ens.spins[a, ja], ens.spins[b, jb])
                    q = rec["q0"][0] + rec["q0"][4] + rec["q0"][8]
                    qr = rec["qk_re"][:, 0] + rec["qk_re"][:, 4] + rec["qk_re"][:, 8]
                    qi = rec["qk_im"][:, 0] + rec["qk_im"][:, 4] + rec["qk_im"][:, 8]
                    q2[k] += q * q / len(pairs)
                    qk2[k] += (qr ** 2 + qi ** 2).mean() / len(pairs)
                    e[k] += (ens.E[a, ja] + ens.E[b, jb]) / (2.0 * N) / len(pairs)
            rows.append((q2, qk2, e))
    last = rows[len(rows) // 2:]
    return {key: np.mean([r[i] for r in last], axis=0) for i, key in enumerate(("q2", "qk2", "e"))}


def test_fss_against_oracle_same_samples():
    """fss.simulate on the GPU against the FP64 oracle on the same disorder
    samples (the same Gaussian couplings, independent random streams), L = 4
    and 8, 16 samples, 6 geometric temperatures in [0.9, 1.6], 2 replicas,
    512 steps of 1 HB + L OR + PT, a measurement every 4 steps, last half
    (Sec. III).  Per sample the two runs differ only by thermal noise, so
    the per-sample differences of <q^2>, <|q(k_min)|^2> and e have mean zero;
    a t statistic over the 16 samples (their spread as the error) is formed
    per (L, temperature, observable).  Rule: every |t| < 4 and at most a
    quarter above 2 (15 degrees of freedom; no error scaling).  The
    disorder-averaged xi/L of the two sides are printed beside it."""
    import concurrent.futures as cf
    import os
    temps = inputs.geometric_temps(0.9, 1.6, 6)
    S, R, steps, every, seed, oseed = 16, 2, 512, 4, 3301, 93301
    ts = []
    for L in (4, 8):
        run = fss.simulate(L, S, temps, R, steps, every, seed, "gaussian", log=lambda m: None)
        gpu = {k: np.asarray(run["means"][k])[0] for k in ("q2", "qk2", "e")}
        cpl = [inputs.gaussian_couplings(L, seed, s) for s in range(S)]
        with cf.ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as pool:
            orc = list(pool.map(lambda s: _oracle_run(L, cpl[s], temps, R, steps, every, oseed, s), range(S)))
        orc = {k: np.stack([o[k] for o in orc]) for k in ("q2", "qk2", "e")}
        for k in ("q2", "qk2", "e"):
            d = gpu[k] - orc[k]
            t = d.mean(axis=0) / (d.std(axis=0, ddof=1) / np.sqrt(S))
            ts.append(t)
            print(f"L={L} {k}: t = {np.round(t, 2)}", flush=True)
        xg, xo = _xi_over_L(gpu, L), _xi_over_L(orc, L)
        print(f"L={L} xi/L gpu {np.round(xg, 3)} oracle {np.round(xo, 3)}", flush=True)
    ts = np.concatenate(ts)
    assert np.all(np.isfinite(ts)), ts
    assert np.all(np.abs(ts) < 4), ts
    assert np.mean(np.abs(ts) > 2) <= 0.25, ts


def _xi_over_L(means, L):
    """xi/L per temperature from the sample-averaged <q^2> and <|q(k_min)|^2>."""
    return A.xi_second_moment(means["q2"].mean(axis=0), means["qk2"].mean(axis=0), L) / L
