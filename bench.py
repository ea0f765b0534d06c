"""Benchmark: picoseconds per spin update of the whole Monte Carlo step on
one MI355X, with the HBM roofline of the dominant kernel and the FP64 oracle
timed beside it.

Workload (default): L = 64, 8 disorder samples, 32 temperatures x 4
replicas = 1024 chains, Gaussian 3x3 couplings; one step = 1 heat-bath +
64 overrelaxation sweeps + 1 tempering pass, with the overlap / chirality /
Schwinger-Dyson measurement every 10 steps.  Inputs are resident in HBM
before the timed region.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 78.6     # non-packed FP32 FMA: 256 CUs x 64 lanes x 2 flops x 2.4 GHz
FLOPS_PER_SU = 138
METRIC = "ps per spin update (all chains) & HBM roofline %, batched FP32 vs plain FP64"
KERNEL_SOURCES = ["paper_1309_1599_amd/csrc/sweep.hip", "paper_1309_1599_amd/csrc/sweep_cl.hip",
                  "paper_1309_1599_amd/csrc/sweep_rs.hip",
                  "paper_1309_1599_amd/csrc/spin_update.hpp", "paper_1309_1599_amd/csrc/kernels.hpp",
                  "paper_1309_1599_amd/csrc/philox.hpp"]
PMC_SUMMARY = os.path.join(ROOT, "profiles", "overrelax_half_sweep_L64x8_pmc.txt")


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_traffic(expected_hash):
    """HBM bytes per overrelaxation launch from the committed rocprofv3 --pmc
    summary, if it was taken on the current kernel source."""
    try:
        text = open(PMC_SUMMARY).read()
    except OSError:
        return None
    m = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", text)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not b or m.group(1) != expected_hash:
        return None
    return float(b.group(1))


def cpu_baseline(L, cpl, temps, seed, n_chains=64, n_or=12):
    """The FP64 oracle as it stands, single-threaded, on a bounded sample of
    the same workload: n_chains chains of sample 0, one heat-bath sweep,
    n_or overrelaxation sweeps and one energy evaluation each; the step's
    per-spin-update time is composed with the real step's weights."""
    import oracle as O
    N = L ** 3
    M = cpl.astype(np.float64)
    t_hb = t_or = t_e = 0.0
    for c in range(n_chains):
        k, r = c % len(temps), c // len(temps)
        s = O.init_spins(L, seed, 0, k, r)
        t0 = time.perf_counter()
        O.sweep(L, M, s, 1, 1.0 / temps[k], seed, 0, 0, k, r)
        t1 = time.perf_counter()
        for _ in range(n_or):
            O.sweep(L, M, s, 0, 1.0 / temps[k], seed, 0, 0, k, r)
        t2 = time.perf_counter()
        O.energy(L, M, s)
        t3 = time.perf_counter()
        t_hb += t1 - t0
        t_or += t2 - t1
        t_e += t3 - t2
    per_hb = t_hb / (n_chains * N)
    per_or = t_or / (n_chains * n_or * N)
    per_e = t_e / n_chains
    return per_hb, per_or, per_e, t_hb + t_or + t_e


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--preset", default="L64x8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every kernel of a step instead of replaying a captured hipGraph")
    ap.add_argument("--mapping", choices=("auto", "site", "chain", "resident"), default="auto",
                    help="sweep kernel mapping (auto: resident for L <= 16, else chain lanes when "
                         "a sample's chains fill 64-lane waves to >= 90%%)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path does not "
              f"span GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1309_1599_amd import inputs, ptsg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    p = inputs.PRESETS[args.preset]
    Ls, cpl, temps, R, seed = inputs.preset_inputs(args.preset)
    n_hb = p["n_hb"]
    n_or_of = (lambda L: L) if p["n_or"] is None else (lambda L: p["n_or"])
    assert len(set(Ls)) == 1, "bench times one lattice size per run"
    L = Ls[0]
    n_or = n_or_of(L)
    every = p["measure_every"]

    # plain copy of a known size: calibrates the rocprofv3 byte counters
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    del a, b

    flags = {"auto": 0, "site": ptsg.PT_F_SITE_LANES, "chain": ptsg.PT_F_CHAIN_LANES,
             "resident": ptsg.PT_F_RESIDENT}[args.mapping]
    C_sample = R * len(temps[0])
    if args.mapping != "auto":
        mapping = args.mapping
    elif L <= 16:
        mapping = "resident"
    else:
        waves = (C_sample + 63) // 64
        mapping = "chain" if L <= 128 and 10 * C_sample >= 9 * 64 * waves else "site"
    if not args.no_graphs:
        flags |= ptsg.PT_F_GRAPHS
    ctx = ptsg.pt_init_batch(Ls, cpl, temps, R, seed, flags=flags)
    n_chains = ctx.n_chains
    N = L ** 3
    su_per_step = (n_hb + n_or) * n_chains * N

    def step(t):
        ptsg.pt_step(ctx, n_hb, n_or)
        ptsg.pt_swap(ctx)
        if every and (t + 1) % every == 0:
            ptsg.pt_measure(ctx, ptsg.PT_M_ALL)

    for t in range(args.warmup):
        step(t)
    ptsg.pt_sync(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(args.steps):
        step(t)
    ptsg.pt_sync(ctx)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # Kernel durations: the same steps again with the dispatches stamping HIP
    # events (kernel start and end, on the library's stream); these steps run
    # without the captured graph and are not part of `value`.
    ptsg.pt_profile(ctx, True)
    for t in range(args.steps):
        step(t)
    ptsg.pt_sync(ctx)
    n_or_launch, or_ms = ptsg.pt_kernel_time(ctx, ptsg.PT_K_OVERRELAX)
    n_hb_launch, hb_ms = ptsg.pt_kernel_time(ctx, ptsg.PT_K_HEATBATH)
    n_rs_launch, rs_ms = ptsg.pt_kernel_time(ctx, ptsg.PT_K_RESIDENT)
    ptsg.pt_profile(ctx, False)

    ps_per_su = wall / (args.steps * su_per_step) * 1e12
    C = R * len(temps[0])
    if mapping != "resident":
        # HBM roofline of the overrelaxation half-sweep: per spin update the
        # method must read and write the spin (24 B) and read the couplings
        # of the site (108 B), which the C chains of a sample share
        bytes_per_su = 24.0 + 108.0 / C
        or_su = args.steps * n_or * n_chains * N       # over all launches of the timed region
        su_per_launch = or_su / max(1, n_or_launch)
        avg_s = or_ms / max(1, n_or_launch) / 1e3
        achieved = bytes_per_su * su_per_launch / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": ("cl_half_sweep_kernel<overrelax>" if mapping == "chain"
                                           else "half_sweep_kernel<overrelax>"),
                "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": pmc_traffic(kernel_hash()),
                "algorithmic_bytes_per_launch": bytes_per_su * su_per_launch,
                "bytes_per_su": round(bytes_per_su, 4), "avg_launch_ms": round(avg_s * 1e3, 4),
                "launches": n_or_launch}
    else:
        # the lattice stays in LDS for the whole step: bounded by FP32 vector
        # arithmetic, 138 flops per overrelaxation update (54-term field,
        # reflection, renormalisation); packed FP32 is not used
        su_per_launch = su_per_step * args.steps / max(1, n_rs_launch)
        avg_s = rs_ms / max(1, n_rs_launch) / 1e3
        achieved = FLOPS_PER_SU * su_per_launch / avg_s / 1e12
        roof = {"bound": "alu", "kernel": "resident_step_kernel", "achieved": round(achieved, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": None, "flops_per_su": FLOPS_PER_SU, "avg_launch_ms": round(avg_s * 1e3, 4),
                "launches": n_rs_launch}
    roof["kernel_source_sha256"] = kernel_hash()

    result = {
        "metric": METRIC,
        "value": round(ps_per_su, 4),
        "unit": "ps/SU",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.preset}: L={L}, {len(Ls)} samples x {len(temps[0])} temperatures x "
                        f"{R} replicas = {n_chains} chains, Gaussian 3x3 couplings; step = {n_hb} HB + "
                        f"{n_or} OR sweeps + PT pass" + (f", measurement every {every} steps" if every else ""),
            "L": L, "samples": len(Ls), "temperatures": len(temps[0]), "replicas": R,
            "spin_updates_per_step": su_per_step,
            "mapping": mapping + " lanes",
            "graphs": not args.no_graphs,
        },
        "roofline": roof,
        "heatbath_avg_launch_ms": round(hb_ms / max(1, n_hb_launch), 4),
    }
    if not args.no_cpu_baseline:
        per_hb, per_or, per_e, spent = cpu_baseline(L, cpl[0], temps[0], seed)
        step_s = (n_hb * per_hb + n_or * per_or) * N + per_e
        result["cpu_baseline"] = {
            "value": round(step_s / ((n_hb + n_or) * N) * 1e12, 1),
            "unit": "ps/SU",
            "cores": 1,
            "kind": "oracle",
            "sample": f"64 chains of sample 0 at L={L}: 1 heat-bath + 12 overrelaxation sweeps and one "
                      f"energy each ({spent:.1f} s), composed to the {n_hb} HB + {n_or} OR step",
        }
    print(json.dumps(result), flush=True)
    ptsg.pt_free(ctx)


if __name__ == "__main__":
    main()
