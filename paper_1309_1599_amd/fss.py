"""Finite-size-scaling runs on the library (Sec. III, Sec. IV).

`simulate` runs one lattice size: a batch of disorder samples, each with
N_T temperatures x R replicas, the paper's Monte Carlo step (1 heat-bath +
L overrelaxation sweeps + 1 tempering pass) for a number of steps, and a
measurement every few steps.  Per (sample, temperature slot) it keeps, for
every logarithmic bin of the measurement series (the last half, the
quarter before it, ...), the sums of q^2 and |q(k_min)|^2 of the scalar
spin-glass overlap (and, with chiral=True, of the chiral-glass overlap
averaged over mu) over the measurements and replica pairs of the bin, and
per sample the autocorrelation time of the temperature random walk of its
chains (Sec. III).

`analyse` turns two such runs (L and bL on one temperature grid, b = 2 in
the paper) into xi_L/L and xi_bL/(bL) of either channel from the last bin,
with jackknife errors over samples (the correlation length is computed from
the disorder-averaged susceptibilities, Sec. II.B): their crossing
temperature from linear fits to the four temperatures nearest to it, xi/L
there, nu from the ratio of the slopes of xi and eta from the ratio of the
susceptibilities (the quotient method of Sec. IV).  `report` adds the
thermalisation test of Sec. III on chi(0) per bin and the walk times.

Run as  python -m paper_1309_1599_amd.fss --L 8 16 --samples 256 ...
(--save FILE.npz keeps the per-sample bin means; --combine A.npz B.npz ...
analyses several such runs of independent samples together.)
"""
import argparse
import json
import sys
import time

import numpy as np

from . import analysis as A
from . import inputs, ptsg


def simulate(L, n_samples, temps, R, steps, measure_every, seed, couplings="bimodal", D=1.0,
             flags=ptsg.PT_F_GRAPHS | ptsg.PT_F_AUTOTUNE, chiral=False, log=print):
    temps = np.asarray(temps, dtype=np.float64)
    T = len(temps)
    if couplings == "bimodal":
        cpl = [inputs.bimodal_couplings(L, D, seed, s) for s in range(n_samples)]
        flags |= ptsg.PT_F_BIMODAL
    else:
        cpl = [inputs.gaussian_couplings(L, seed, s) for s in range(n_samples)]
    ctx = ptsg.pt_init_batch([L] * n_samples, cpl, [temps] * n_samples, R, seed, flags=flags)
    del cpl
    n_meas = steps // measure_every
    bins = A.log_bins(n_meas)
    which = np.full(n_meas, -1)
    for i, (lo, hi) in enumerate(bins):
        which[lo:hi] = i
    nb = len(bins)
    keys = ("q2", "qk2", "e") + (("cg2", "cgk2") if chiral else ())
    what = ptsg.PT_M_OVERLAP | (ptsg.PT_M_CHIRAL if chiral else 0)
    sums = {k: np.zeros((nb, n_samples, T)) for k in keys}
    counts = np.zeros(nb)
    walk = np.empty((n_meas, n_samples, R * T), np.int16)   # slot of every chain at each measurement
    t0 = time.perf_counter()
    m = 0
    for step in range(1, steps + 1):
        ptsg.pt_step(ctx, 1, L)
        ptsg.pt_swap(ctx)
        if step % measure_every == 0:
            recs = ptsg.pt_measure(ctx, what)
            walk[m] = A.slot_of_chain(np.stack(ptsg.pt_get_perms(ctx))).reshape(n_samples, R * T)
            b = which[m]
            if b >= 0:
                F = A.fields(recs[None], L)
                s, k = recs["sample"], recs["tslot"]
                for key in sums:
                    np.add.at(sums[key][b], (s, k), F[key][0])
                counts[b] += 1
            m += 1
        if step % max(1, steps // 20) == 0:
            log(f"L={L}: step {step}/{steps} ({time.perf_counter() - t0:.0f} s)")
    pairs = R * (R - 1) // 2
    ptsg.pt_free(ctx)
    means = {k: v / (counts[:, None, None] * pairs) for k, v in sums.items()}
    # Sec. III: autocorrelation time of each sample's temperature walk over
    # the last half of the run, in Monte Carlo steps
    tau = [A.temperature_walk_tau(walk[n_meas // 2:, s]) * measure_every for s in range(n_samples)]
    return {"L": L, "temps": temps.tolist(), "R": R, "steps": steps, "measure_every": measure_every,
            "n_samples": n_samples, "bins": bins, "counts": counts.tolist(),
            "means": {k: v.tolist() for k, v in means.items()}, "tau_walk": tau,
            "seconds": time.perf_counter() - t0}


CHANNELS = {"sg": ("q2", "qk2"), "cg": ("cg2", "cgk2")}


def _blocks(run, b=0, channel="sg"):
    """(n_samples, 2, T) per-sample chi(0), chi(k_min) of bin b (0 = last)
    for the spin-glass ("sg") or chiral-glass ("cg") overlap."""
    N = run["L"] ** 3
    k0, kk = CHANNELS[channel]
    q2 = np.asarray(run["means"][k0])[b]
    qk2 = np.asarray(run["means"][kk])[b]
    return np.stack([N * q2, N * qk2], axis=1)


def xi_over_L(run, b=0, channel="sg"):
    """xi/L per temperature from the disorder-averaged susceptibilities of
    bin b, with jackknife errors over samples."""
    L = run["L"]
    return A.jackknife(_blocks(run, b, channel), lambda m: A.xi_second_moment(m[0], m[1], L) / L)


def analyse(small, large, n_fit=4, extrapolate=0.25, channel="sg"):
    """Crossing of xi/L between two runs on one temperature grid (linear
    fits to the four temperatures nearest to it; a crossing up to a quarter
    of the grid's width beyond its edge is extrapolated and flagged)."""
    T = np.asarray(small["temps"])
    assert np.allclose(T, large["temps"]), "the two sizes need one temperature grid"
    n = min(small["n_samples"], large["n_samples"])
    Ls, Ll = small["L"], large["L"]
    b1, b2 = _blocks(small, 0, channel)[:n], _blocks(large, 0, channel)[:n]   # sample i of each size forms block i

    b = Ll / Ls

    def f(m):
        y1 = A.xi_second_moment(m[0], m[1], Ls) / Ls
        y2 = A.xi_second_moment(m[2], m[3], Ll) / Ll
        tc, yc, s1, s2 = A.crossing(T, y1, y2, n_fit=n_fit, extrapolate=extrapolate)
        # quotients at the crossing (Sec. IV): d xi/dT = L d(xi/L)/dT, and chi(0)
        # of both sizes from the same local linear fits
        ratio_chi = A.value_at(T, m[2], tc, n_fit) / A.value_at(T, m[0], tc, n_fit)
        return np.array([tc, yc, (Ll * s2) / (Ls * s1), A.eta_from_chi_ratio(ratio_chi, b)])

    est, err = A.jackknife(np.concatenate([b1, b2], axis=1), f)
    out = {"channel": channel, "pair": [Ls, Ll], "T_cross": [est[0], err[0]], "xi_over_L_cross": [est[1], err[1]],
           "slope_ratio": [est[2], err[2]], "eta": [est[3], err[3]],
           "extrapolated": bool(est[0] < T.min() or est[0] > T.max())}
    if est[2] > b:
        nu = A.nu_from_slope_ratio(est[2], b)
        # error of nu from the jackknife of the ratio (propagated)
        lr = np.log(est[2]) / np.log(b)
        dnu = err[2] / (est[2] * np.log(b) * (lr - 1) ** 2)
        out["nu"] = [nu, dnu]
    return out


def thermalisation(run):
    """Sec. III test on chi_SG(0): per logarithmic bin (last first), the
    disorder average of chi(0) minus that of the last bin, per temperature,
    with jackknife errors over samples."""
    N = run["L"] ** 3
    q2 = N * np.asarray(run["means"]["q2"])        # (bins, samples, T)
    out = []
    for b in range(q2.shape[0]):
        if run["counts"][b] == 0:
            continue
        d = q2[b] - q2[0]
        m, e = A.jackknife(d)
        out.append({"bin": run["bins"][b], "diff": m.tolist(), "err": e.tolist()})
    return out


def save_runs(path, runs):
    """Per-sample bin means of every run, for combining batches later."""
    arrays = {}
    for r in runs:
        L = r["L"]
        for k, v in r["means"].items():
            arrays[f"L{L}_{k}"] = np.asarray(v)
        arrays[f"L{L}_temps"] = np.asarray(r["temps"])
        arrays[f"L{L}_counts"] = np.asarray(r["counts"])
        arrays[f"L{L}_bins"] = np.asarray(r["bins"])
        arrays[f"L{L}_meta"] = np.asarray([r["R"], r["steps"], r["measure_every"], r["n_samples"]])
        if "tau_walk" in r:
            arrays[f"L{L}_tau_walk"] = np.asarray(r["tau_walk"])
    np.savez(path, **arrays)


def load_runs(paths):
    """Runs of the same sizes from several saved batches, samples concatenated."""
    runs = {}
    for path in paths:
        z = np.load(path)
        for L in sorted({int(k.split("_")[0][1:]) for k in z.files}):
            means = {k: z[f"L{L}_{k}"] for k in ("q2", "qk2", "e", "cg2", "cgk2") if f"L{L}_{k}" in z.files}
            meta = z[f"L{L}_meta"]
            if L not in runs:
                runs[L] = {"L": L, "temps": z[f"L{L}_temps"].tolist(), "R": int(meta[0]), "steps": int(meta[1]),
                           "measure_every": int(meta[2]), "n_samples": 0, "bins": z[f"L{L}_bins"].tolist(),
                           "counts": z[f"L{L}_counts"].tolist(), "means": {k: [] for k in means}}
            r = runs[L]
            assert np.allclose(r["temps"], z[f"L{L}_temps"]) and r["steps"] == int(meta[1])
            for k, v in means.items():
                r["means"][k].append(v)
            r.setdefault("tau_parts", []).append(z[f"L{L}_tau_walk"] if f"L{L}_tau_walk" in z.files else None)
            r["n_samples"] += int(meta[3])
    for r in runs.values():
        r["means"] = {k: np.concatenate(v, axis=1) for k, v in r["means"].items()}
        parts = r.pop("tau_parts")
        if all(t is not None for t in parts):
            r["tau_walk"] = np.concatenate(parts).tolist()
    return [runs[L] for L in sorted(runs)]


def walk_summary(run):
    """Sec. III criterion: the temperature-walk autocorrelation times of the
    samples (MCS) and the share of samples whose run is at least 10 of them."""
    tau = np.asarray(run["tau_walk"], dtype=np.float64)
    return {"median": float(np.median(tau)), "max": float(tau.max()),
            "runs_longer_than_10_tau": float(np.mean(run["steps"] >= 10 * tau))}


def report(runs, temps, couplings, D):
    channels = ["sg"] + (["cg"] if all("cg2" in r["means"] for r in runs) else [])
    result = {"runs": [{k: r[k] for k in ("L", "n_samples", "steps") if k in r} for r in runs],
              "temps": list(map(float, temps)), "couplings": couplings, "D": D,
              "xi_over_L": {str(r["L"]): [v.tolist() for v in xi_over_L(r)] for r in runs},
              "thermalisation_chi0": {str(r["L"]): thermalisation(r) for r in runs},
              "temperature_walk": {str(r["L"]): walk_summary(r) for r in runs if "tau_walk" in r},
              "crossings": []}
    if "cg" in channels:
        result["xi_cg_over_L"] = {str(r["L"]): [v.tolist() for v in xi_over_L(r, 0, "cg")] for r in runs}
    for ch in channels:
        for a, b in zip(runs, runs[1:]):
            try:
                result["crossings"].append(analyse(a, b, channel=ch))
            except ValueError as e:
                result["crossings"].append({"channel": ch, "pair": [a["L"], b["L"]], "error": str(e)})
    return result


def make_parser():
    """The command line; its defaults are the paper's D = 1 protocol at L = 8
    and 16 (Table I), on one 28-temperature grid for both sizes."""
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--L", type=int, nargs="+", default=[8, 16])
    ap.add_argument("--samples", type=int, default=256)
    ap.add_argument("--steps", type=int, nargs="+", default=[20480, 40960],
                    help="Monte Carlo steps per size (one value, or one per size)")
    ap.add_argument("--temps", type=float, nargs=3, default=[0.877, 1.28, 28], metavar=("TMIN", "TMAX", "N"))
    ap.add_argument("--replicas", type=int, default=2)
    ap.add_argument("--measure-every", type=int, default=10)
    ap.add_argument("--couplings", choices=("bimodal", "gaussian"), default="bimodal")
    ap.add_argument("--D", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=1309)
    ap.add_argument("--chiral", action="store_true", help="also measure the chiral-glass overlap (Sec. II.B)")
    ap.add_argument("--out", default=None)
    ap.add_argument("--save", default=None, help="write per-sample bin means (npz)")
    ap.add_argument("--combine", nargs="+", default=None, help="analyse saved batches together (no GPU)")
    return ap


def main(argv=None):
    args = make_parser().parse_args(argv)
    if args.combine:
        runs = load_runs(args.combine)
        result = report(runs, runs[0]["temps"], args.couplings, args.D)
        if args.out:
            with open(args.out, "w") as fh:
                fh.write(json.dumps(result, default=float))
        print(json.dumps({"samples": [r["n_samples"] for r in runs], "crossings": result["crossings"]},
                         default=float))
        return
    import torch
    torch.cuda.set_device(0)
    temps = inputs.geometric_temps(args.temps[0], args.temps[1], int(args.temps[2]))
    steps = args.steps * len(args.L) if len(args.steps) == 1 else args.steps
    runs = []
    for L, n in zip(args.L, steps):
        runs.append(simulate(L, args.samples, temps, args.replicas, n, args.measure_every,
                             args.seed + L, args.couplings, args.D, chiral=args.chiral,
                             log=lambda msg: print(msg, file=sys.stderr, flush=True)))
    if args.save:
        save_runs(args.save, runs)
    result = report(runs, temps, args.couplings, args.D)
    result["seconds"] = {str(r["L"]): r["seconds"] for r in runs}
    text = json.dumps(result, default=float)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text)
    print(json.dumps(result["crossings"], default=float))


if __name__ == "__main__":
    main()
