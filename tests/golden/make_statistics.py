"""Write tests/golden/statistics_<config>.json: long-run averages of the FP64
oracle over independent runs, the reference side of the long-run
statistical parity test (tests/test_gpu_statistics.py).

Calls only the oracle (oracle/) and the seeded input generators.

Why independent runs.  The GPU library and the oracle simulate the same
Markov chain (the paper's Monte Carlo step, Sec. III: one heat-bath sweep,
L overrelaxation sweeps and one tempering pass; App. A.1) from the same
initial law (hot start).  Any statistic of a run of fixed length therefore
has the same distribution on both sides, whether or not the run has
equilibrated.  Comparing means over independent runs, with errors from the
spread between runs, is exact in that sense: metastable runs at the lowest
temperatures (a replica pair trapped in different valleys for a whole run)
widen the spread instead of biasing the comparison.

Per run and temperature slot, over the second half of the measurements
(one after every step's tempering pass): the energy per spin (both
replicas), <q^2>, <q^4> of the scalar overlap q = tr Q(0) and
<|q(k_min)|^2> averaged over the three directions (Sec. II.B).

Configurations (the parity workloads of the hot path):
  L8:  L = 8, 8 temperatures evenly spaced in [0.5, 2.0], 2 replicas,
       1000 steps of 1 HB + 8 OR + PT; 64 runs.
  L16: L = 16, 16 geometric temperatures in [0.5, 2.0], 2 replicas,
       10^4 steps of 1 HB + 16 OR + PT; 32 runs.
Couplings: the presets' (inputs.preset_inputs), one sample shared by all
runs.  Run i draws its random numbers as sample i of seed ORACLE_SEED (the
GPU side uses the presets' seed: independent streams).

The GPU side of the test runs `gpu_runs` runs (GPU runs cost little, so
more of them shrink the GPU share of the error).

Usage: python tests/golden/make_statistics.py L8 [L16] [--procs 8] [--extend]
(--extend keeps the runs already in the file and adds the missing ones:
run i depends only on i.)
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CONFIGS = {
    "L8": dict(preset="L8", L=8, steps=1000, runs=64, gpu_runs=64),
    "L16": dict(preset="L16", L=16, steps=10000, runs=32, gpu_runs=64),
}
ORACLE_SEED = 7130915990
OBSERVABLES = ("e", "q2", "q4", "qk2")


def record_fields(q0, qk_re, qk_im, E_a, E_b, L):
    """Per-record observables from the overlap tensor Q(0), the three
    Q(k_min) and the two replicas' energies."""
    tr = lambda a: a[..., 0] + a[..., 4] + a[..., 8]
    q = tr(q0)
    return {"e": (E_a + E_b) / (2.0 * L ** 3), "q2": q ** 2, "q4": q ** 4,
            "qk2": (tr(qk_re) ** 2 + tr(qk_im) ** 2).mean(axis=-1)}


def run_means(fields_per_meas, slots, T):
    """Means over the second half of a run, per slot (pairs of a slot
    averaged).  fields_per_meas: list over measurements of dicts of arrays
    over records; slots: slot of each record."""
    n = len(fields_per_meas)
    keep = fields_per_meas[n // 2:]
    out = {}
    for k in OBSERVABLES:
        v = np.mean([f[k] for f in keep], axis=0)
        out[k] = np.bincount(slots, weights=v, minlength=T) / np.bincount(slots, minlength=T)
    return out


def _one_run(args):
    name, i = args
    import oracle as O
    from oracle import OracleEnsemble
    from paper_1309_1599_amd import inputs
    c = CONFIGS[name]
    Ls, cpl, temps, R, _seed = inputs.preset_inputs(c["preset"])
    L, T = Ls[0], len(temps[0])
    ens = OracleEnsemble(L, cpl[0], temps[0], R, ORACLE_SEED, sample=i)
    pairs = [(k, a, b) for k in range(T) for a in range(R) for b in range(a + 1, R)]
    slots = np.array([p[0] for p in pairs])
    meas = []
    for _ in range(c["steps"]):
        ens.step(1, L)
        ens.swap()
        q0, qr, qi, Ea, Eb = [], [], [], [], []
        for (k, a, b) in pairs:
            ja, jb = int(ens.perm[a, k]), int(ens.perm[b, k])
            rec = O.overlaps(L, ens.spins[a, ja], ens.spins[b, jb])
            q0.append(rec["q0"]); qr.append(rec["qk_re"]); qi.append(rec["qk_im"])
            Ea.append(ens.E[a, ja]); Eb.append(ens.E[b, jb])
        meas.append(record_fields(np.array(q0), np.array(qr), np.array(qi), np.array(Ea), np.array(Eb), L))
    m = run_means(meas, slots, T)
    return {k: v.tolist() for k, v in m.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("configs", nargs="+", choices=list(CONFIGS))
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--extend", action="store_true")
    a = ap.parse_args()
    for name in a.configs:
        c = CONFIGS[name]
        path = os.path.join(HERE, f"statistics_{name}.json")
        runs = []
        if a.extend and os.path.exists(path):
            with open(path) as f:
                old = json.load(f)
            if old["steps"] == c["steps"] and old["oracle_seed"] == ORACLE_SEED:
                runs = old["runs"][:c["runs"]]
        t0 = time.time()
        with mp.get_context("spawn").Pool(a.procs) as pool:
            runs += pool.map(_one_run, [(name, i) for i in range(len(runs), c["runs"])], chunksize=1)
        out = dict(config=name, preset=c["preset"], L=c["L"], steps=c["steps"], n_runs=c["runs"],
                   oracle_seed=ORACLE_SEED, observables=list(OBSERVABLES),
                   note="second-half means per run and slot; written by tests/golden/make_statistics.py "
                        "from the FP64 oracle only",
                   runs=runs)
        with open(path, "w") as f:
            json.dump(out, f, indent=0)
        print(f"{name}: {c['runs']} runs in {time.time() - t0:.0f} s -> {path}", flush=True)


if __name__ == "__main__":
    main()
