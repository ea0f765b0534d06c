"""Long-run statistical parity: the GPU and the FP64 oracle simulate the same
sample (same couplings and temperatures) with independent random streams,
and the equilibrium averages must agree within their errors.

Workload: L = 8, 8 temperatures evenly spaced in [0.7, 2.0], 2 replicas;
each step = 1 heat-bath + 8 overrelaxation sweeps + 1 tempering pass, the
paper's Monte Carlo step (Sec. III); measurements after every step.
Observables per temperature: energy per spin, <q^2>, <q^4> of the scalar
overlap q = tr Q(0), and the second-moment correlation length of Sec. II.B
(Eq. for xi with k_min = 2 pi / L along each axis).  The first half of each
run is discarded; errors from 16 blocks.  Rule: every |z| < 4 and at most a
quarter of the |z| above 2.  (Nothing in the paper fixes these values for
Gaussian couplings; the pin is GPU-versus-oracle agreement.)

Calibration, from the oracle alone: eight runs with independent seeds gave
pairwise z-scores with an rms of 1.34 (the 16-block errors miss part of the
autocorrelation), so the errors are scaled by ERR_SCALE = 1.5.  The lowest
temperature is 0.7 because at 0.5 two of four oracle seeds stayed in a
metastable state (q^2 near 0.07 against 0.53) for the whole run: that
temperature is not equilibrated in 2000 steps and no parity can be read
from it.
"""
import numpy as np
import pytest

from oracle import OracleEnsemble
from paper_1309_1599_amd import inputs, ptsg

pytestmark = pytest.mark.gpu

L, T, R, STEPS = 8, 8, 2, 2000
T_MIN, ERR_SCALE = 0.7, 1.5
N = L ** 3


def _observables(recs_by_step):
    """recs_by_step: list over steps of arrays/dicts with q0, qk_re, qk_im,
    E_a, E_b per (slot) for the pair (0, 1)."""
    out = {k: [] for k in ("e", "q2", "q4", "chi0", "chik")}
    for recs in recs_by_step:
        q = np.array([np.trace(np.asarray(r["q0"]).reshape(3, 3)) for r in recs])
        qk = np.array([[np.trace(np.asarray(r["qk_re"])[d].reshape(3, 3)) ** 2
                        + np.trace(np.asarray(r["qk_im"])[d].reshape(3, 3)) ** 2 for d in range(3)]
                       for r in recs]).mean(axis=1)
        out["e"].append(np.array([(r["E_a"] + r["E_b"]) / (2 * N) for r in recs]))
        out["q2"].append(q ** 2)
        out["q4"].append(q ** 4)
        out["chi0"].append(N * q ** 2)
        out["chik"].append(N * qk)
    return {k: np.array(v) for k, v in out.items()}


def _blocks(obs, nb=16):
    h = len(obs["e"]) // 2
    res = {}
    for k, v in obs.items():
        v = v[h:]
        v = v[: len(v) // nb * nb].reshape(nb, -1, v.shape[1]).mean(axis=1)
        res[k] = v
    return res


def _stats(b):
    """means and jackknife errors per slot of e, q2, q4, xi/L"""
    nb = b["e"].shape[0]
    def xi(chi0, chik):
        ratio = np.maximum(chi0 / chik - 1.0, 0.0)
        return np.sqrt(ratio) / (2 * np.sin(np.pi / L)) / L
    means, errs = {}, {}
    for k in ("e", "q2", "q4"):
        means[k] = b[k].mean(axis=0)
        errs[k] = b[k].std(axis=0, ddof=1) / np.sqrt(nb)
    full = xi(b["chi0"].mean(axis=0), b["chik"].mean(axis=0))
    jk = np.array([xi(np.delete(b["chi0"], i, 0).mean(axis=0), np.delete(b["chik"], i, 0).mean(axis=0))
                   for i in range(nb)])
    means["xi"] = full
    errs["xi"] = np.sqrt((nb - 1) / nb * ((jk - jk.mean(axis=0)) ** 2).sum(axis=0))
    return means, errs


def test_long_run_statistics_match_oracle():
    temps = inputs.linear_temps(T_MIN, 2.0, T)
    cpl = inputs.gaussian_couplings(L, 130915991)
    # GPU run
    ctx = ptsg.pt_init_batch([L], [cpl], [temps], R, 1001)
    gpu = []
    for _ in range(STEPS):
        ptsg.pt_step(ctx, 1, L)
        ptsg.pt_swap(ctx)
        gpu.append(ptsg.pt_measure(ctx, ptsg.PT_M_OVERLAP))
    ptsg.pt_free(ctx)
    # oracle run, independent seed
    ens = OracleEnsemble(L, cpl, temps, R, 2002)
    orc = []
    for _ in range(STEPS):
        ens.step(1, L)
        ens.swap()
        orc.append(ens.measure())
    mg, eg = _stats(_blocks(_observables(gpu)))
    mo, eo = _stats(_blocks(_observables(orc)))
    zs = []
    for k in ("e", "q2", "q4", "xi"):
        z = (mg[k] - mo[k]) / (ERR_SCALE * np.sqrt(eg[k] ** 2 + eo[k] ** 2) + 1e-300)
        zs.append(z)
        print(k, np.round(mg[k], 4), np.round(mo[k], 4), np.round(z, 2))
    zs = np.concatenate(zs)
    assert np.all(np.abs(zs) < 4), zs
    assert np.mean(np.abs(zs) > 2) <= 0.25, zs
