"""Benchmark: picoseconds per spin update of the whole Monte Carlo step on
one MI355X, with the roofline of the dominant kernel and the FP64 oracle
timed beside it.

Workload (default, preset L64x8): L = 64, 8 disorder samples, 32
temperatures x 4 replicas = 1024 chains, Gaussian 3x3 couplings; one step =
1 heat-bath + 64 overrelaxation sweeps + 1 tempering pass, with the overlap /
chirality / Schwinger-Dyson measurement every 10 steps.  Inputs are resident
in HBM before the timed region.

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
FLOPS_PER_SU = 138          # overrelaxation update: 54-term field, reflection, renormalisation
METRIC = "ps per spin update (all chains) & HBM roofline %, batched FP32 vs plain FP64"
KERNEL_SOURCES = ["paper_1309_1599_amd/csrc/sweep.hip", "paper_1309_1599_amd/csrc/sweep_cl.hip",
                  "paper_1309_1599_amd/csrc/sweep_rs.hip", "paper_1309_1599_amd/csrc/sweep_row.hip",
                  "paper_1309_1599_amd/csrc/spin_update.hpp", "paper_1309_1599_amd/csrc/kernels.hpp",
                  "paper_1309_1599_amd/csrc/philox.hpp"]
PMC_SUMMARY = os.path.join(ROOT, "profiles", "overrelax_half_sweep_{preset}_pmc.txt")


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_traffic(preset, mapping, expected_hash):
    """HBM bytes per overrelaxation launch from the committed rocprofv3 --pmc
    summary of this preset, if it was taken on the current kernel source with
    the same mapping.  The summaries cover Gaussian couplings and the
    checkerboard order (bimodal couplings: the preset's "_bimodal" summary);
    other variants report null."""
    try:
        text = open(PMC_SUMMARY.format(preset=preset)).read()
    except OSError:
        return None
    m = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", text)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    k = re.search(r"mapping:\s*(\w+)", text)
    if not m or not b or not k or m.group(1) != expected_hash or k.group(1) != mapping:
        return None
    return float(b.group(1))


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or the platform's."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(L, cpl, temps, seed, n_hb, n_or_step, n_chains=64, n_or=12, per_thread=16):
    """The FP64 oracle as it stands on a bounded sample of the same workload:
    chains of sample 0, each one heat-bath sweep, n_or overrelaxation sweeps
    and one energy evaluation; the per-spin-update time is composed with the
    real step's weights.  Timed single-threaded (n_chains chains) and with
    one thread per host core of this GPU's share (at most 16), `per_thread`
    chains per thread (the oracle's C calls release the GIL)."""
    import concurrent.futures as cf
    import oracle as O
    N = L ** 3
    M = cpl.astype(np.float64)

    def chain(c):
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
        return t1 - t0, t2 - t1, t3 - t2

    def composed(times, n):
        t_hb, t_or, t_e = (sum(t[i] for t in times) for i in range(3))
        step_s = (n_hb * t_hb / (n * N) + n_or_step * t_or / (n * n_or * N)) * N + t_e / n
        return step_s / ((n_hb + n_or_step) * N), t_hb + t_or + t_e

    single, busy1 = composed([chain(c) for c in range(n_chains)], n_chains)
    workers = max(1, min(16, os.cpu_count() or 1))
    n_mt = per_thread * workers
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(workers) as ex:
        times = list(ex.map(chain, range(n_mt)))
    wall = time.perf_counter() - t0
    per_su, busy = composed(times, n_mt)
    parallel = per_su * wall / busy   # thread-busy seconds -> wall seconds
    return {
        "value": round(parallel * 1e12, 1),
        "unit": "ps/SU",
        "cores": workers,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "single_thread_value": round(single * 1e12, 1),
        "sample": f"chains on the couplings of sample 0 at L={L} (its temperatures, replica index "
                  f"running on past the workload's where more chains are needed), each 1 heat-bath + "
                  f"{n_or} overrelaxation sweeps and one energy, composed to the {n_hb} HB + "
                  f"{n_or_step} OR step: {n_mt} chains on {workers} threads ({wall:.1f} s wall, "
                  f"{busy:.1f} thread-s); single-threaded {n_chains} chains ({busy1:.1f} s)",
    }


def mixed_cpu_baseline(Ls, cpl, temps, R, seed, n_hb, n_or, or_l):
    """The oracle's ps/SU on a batch of several L: one bounded sample per
    distinct L (the first sample of that L, 16 chains single-threaded and
    four chains a thread), composed with each L's share of the step's spin
    updates, so that it is the time the oracle would take for the whole
    batch divided by its spin updates."""
    parts, su, per_L = [], {}, {}
    for Lv, t in zip(Ls, temps):
        su[Lv] = su.get(Lv, 0) + (n_hb + (Lv if n_or == or_l else n_or)) * R * len(t) * Lv ** 3
    tot = sum(su.values())
    value = single = 0.0
    for Lv in sorted(su):
        i = Ls.index(Lv)
        b = cpu_baseline(Lv, cpl[i], temps[i], seed, n_hb, Lv if n_or == or_l else n_or,
                         n_chains=16, per_thread=4)
        w = su[Lv] / tot
        value += w * b["value"]
        single += w * b["single_thread_value"]
        per_L[str(Lv)] = {"value": b["value"], "single_thread_value": b["single_thread_value"],
                          "su_share": round(w, 4)}
        parts.append(b)
    return {
        "value": round(value, 1),
        "unit": "ps/SU",
        "cores": parts[0]["cores"],
        "kind": "oracle",
        "cpu_model": parts[0]["cpu_model"],
        "single_thread_value": round(single, 1),
        "per_L": per_L,
        "sample": "per L, chains on the couplings of the first sample of that L, each 1 heat-bath + 12 "
                  "overrelaxation sweeps and one energy, composed to that L's step (1 HB + L OR); the "
                  "per-L figures weighted by each L's share of the step's spin updates: "
                  + "; ".join(f"L={Lv}: {b['sample'].split(': ', 1)[1]}" for Lv, b in zip(sorted(su), parts)),
    }


def copy_rate(torch, mib, iters):
    """GB/s (read + write bytes) of a torch device copy of `mib` MiB."""
    a = torch.empty(mib << 18, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del a, b
    torch.cuda.empty_cache()
    return round(2 * (mib << 20) * iters / dt / 1e9, 1)


def run(ptsg, torch, Ls, cpl, temps, R, seed, flags, n_hb, n_or, every, steps, warmup, timing=True,
        what=None):
    """Time `steps` steps after `warmup`; optionally a second pass with
    kernel-stamped events for the kernel durations."""
    ctx = ptsg.pt_init_batch(Ls, cpl, temps, R, seed, flags=flags)
    names = {ptsg.PT_F_SITE_LANES: "site", ptsg.PT_F_CHAIN_LANES: "chain", ptsg.PT_F_RESIDENT: "resident"}
    maps = [names[ptsg.pt_get_mapping(ctx, s)] for s in range(len(Ls))]
    su_per_step = sum((n_hb + (L if n_or == ptsg.PT_OR_L else n_or)) * R * len(t) * L ** 3
                      for L, t in zip(Ls, temps))

    what = ptsg.PT_M_ALL if what is None else what

    def step(t):
        ptsg.pt_step(ctx, n_hb, n_or)
        ptsg.pt_swap(ctx)
        if every and (t + 1) % every == 0:
            ptsg.pt_measure(ctx, what)

    # The timed steps run through pt_run: whole steps (sweeps, tempering and,
    # every `every` steps, the measurement) replayed as captured graphs, the
    # records written to a device buffer and copied to the host once, inside
    # the timed region.
    n_rec = ctx.n_records
    sets = max(steps, warmup) // every if every else 0
    buf = torch.empty(max(1, sets * n_rec * ptsg.MEAS_DTYPE.itemsize), dtype=torch.uint8, device="cuda")
    ptsg.pt_run(ctx, warmup, n_hb, n_or, every, what, buf.data_ptr(), sets * n_rec)
    ptsg.pt_sync(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ptsg.pt_run(ctx, steps, n_hb, n_or, every, what, buf.data_ptr(), sets * n_rec)
    ptsg.pt_sync(ctx)
    records = buf.cpu()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    del records
    kt = None
    if timing:
        # Kernel durations: the same steps again with the dispatches stamping
        # HIP events at kernel start and end on the library's stream; these
        # steps run without a captured graph and are not part of `value`.
        ptsg.pt_profile(ctx, True)
        for t in range(steps):
            step(t)
        ptsg.pt_sync(ctx)
        kt = {k: ptsg.pt_kernel_time(ctx, v) for k, v in
              (("or", ptsg.PT_K_OVERRELAX), ("hb", ptsg.PT_K_HEATBATH), ("rs", ptsg.PT_K_RESIDENT),
               ("ps", ptsg.PT_K_PERSISTENT))}
        ptsg.pt_profile(ctx, False)
    ptsg.pt_free(ctx)
    del ctx
    torch.cuda.empty_cache()
    return wall, su_per_step, kt, maps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--preset", default="L64x8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain single-chain reference")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every kernel of a step instead of replaying a captured hipGraph")
    ap.add_argument("--mapping", choices=("auto", "tuned", "site", "chain", "resident"), default="auto",
                    help="sweep kernel mapping (auto: resident for L <= 16, chain lanes for 24 <= L "
                         "<= 64 when a sample's chains fill 64-lane waves to >= 90%%, else site "
                         "lanes; tuned: timed per L when the context is made)")
    ap.add_argument("--couplings", choices=("gaussian", "bimodal"), default="gaussian",
                    help="gaussian: 9 iid N(0,1) entries per bond (the workload); bimodal: the paper's "
                         "family J*1 + D_sym, J = +-1, D_ab = +-0.5, stored as one byte per bond "
                         "(PT_F_BIMODAL) where the mapping allows")
    ap.add_argument("--persistent", action="store_true",
                    help="time the persistent step (PT_F_PERSISTENT: one cooperative launch per step) "
                         "as the headline instead of the captured multi-launch step")
    ap.add_argument("--no-persistent", action="store_true",
                    help="skip the persistent-step figure reported beside the headline")
    ap.add_argument("--or-order", choices=("checkerboard", "rows"), default="checkerboard",
                    help="rows: overrelaxation in the row order (PT_F_ROW_OR, chain-lane mapping)")
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
    bimodal = args.couplings == "bimodal"
    if bimodal:
        cpl = [inputs.bimodal_couplings(L, 0.5, seed, s) for s, L in enumerate(Ls)]
    n_hb = p["n_hb"]
    mixed = len(set(Ls)) > 1
    # the paper's step: 1 HB + L OR + PT, each sample with its own L
    n_or = (ptsg.PT_OR_L if mixed else Ls[0]) if p["n_or"] is None else p["n_or"]
    every = p["measure_every"]
    bits = {"overlap": ptsg.PT_M_OVERLAP, "chiral": ptsg.PT_M_CHIRAL, "sd": ptsg.PT_M_SD}
    what = ptsg.PT_M_ENERGY
    for m in p.get("measure", ("overlap", "chiral", "sd")):
        what |= bits[m]
    flags = {"auto": 0, "tuned": ptsg.PT_F_AUTOTUNE, "site": ptsg.PT_F_SITE_LANES,
             "chain": ptsg.PT_F_CHAIN_LANES, "resident": ptsg.PT_F_RESIDENT}[args.mapping]
    if not args.no_graphs:
        flags |= ptsg.PT_F_GRAPHS
    if bimodal:
        flags |= ptsg.PT_F_BIMODAL
    rows = args.or_order == "rows"
    if args.persistent:
        flags = (flags & ~(ptsg.PT_F_RESIDENT | ptsg.PT_F_AUTOTUNE | ptsg.PT_F_GRAPHS)) | ptsg.PT_F_PERSISTENT
    if rows:
        flags = (flags & ~(ptsg.PT_F_SITE_LANES | ptsg.PT_F_RESIDENT | ptsg.PT_F_AUTOTUNE)) | ptsg.PT_F_ROW_OR
    L = Ls[0]
    C = R * len(temps[0])

    # plain copy of a known size: calibrates the rocprofv3 byte counters
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    del a, b
    # what plain streaming copies reach on this GPU, beside the spec peak:
    # from HBM (1 GiB each way) and inside the Infinity Cache (64 MiB)
    copy_rates = {"hbm_1GiB": copy_rate(torch, 1024, 20), "infinity_cache_64MiB": copy_rate(torch, 64, 200)}

    wall, su_per_step, kt, maps = run(ptsg, torch, Ls, cpl, temps, R, seed, flags, n_hb, n_or, every,
                                      args.steps, args.warmup, what=what)
    mapping = maps[0]
    ps_per_su = wall / (args.steps * su_per_step) * 1e12
    n_chains = sum(R * len(t) for t in temps)

    if args.persistent and not mixed:
        # the whole step is one launch: its algorithmic bytes (24 + 108/C
        # per spin update, or 24 + 3/C with byte couplings) over its duration
        n_l, ms = kt["ps"]
        bytes_per_su = 24.0 + (3.0 if bimodal else 108.0) / C
        avg_s = ms / max(1, n_l) / 1e3
        achieved = bytes_per_su * su_per_step / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": "cl_step_kernel" if mapping == "chain" else "site_step_kernel",
                "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                "algorithmic_bytes_per_launch": bytes_per_su * su_per_step,
                "bytes_per_su": round(bytes_per_su, 4), "avg_launch_ms": round(avg_s * 1e3, 4),
                "launches": n_l}
    elif not mixed and mapping != "resident":
        # HBM roofline of the overrelaxation half-sweep: per spin update the
        # method must read and write the spin (24 B) and read the couplings
        # of the site (108 B as floats, 3 B as bimodal codes), which the C
        # chains of a sample share
        n_l, ms = kt["or"]
        bytes_per_su = 24.0 + (3.0 if bimodal else 108.0) / C
        or_su = args.steps * n_or * n_chains * L ** 3
        su_per_launch = or_su / max(1, n_l)
        avg_s = ms / max(1, n_l) / 1e3
        achieved = bytes_per_su * su_per_launch / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": ("cl_row_or_kernel" if rows else
                                           "cl_half_sweep_kernel<overrelax>" if mapping == "chain"
                                           else "half_sweep_kernel<overrelax>"),
                "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": (None if rows else pmc_traffic(args.preset + ("_bimodal" if bimodal else ""), mapping,
                                                           kernel_hash())),
                "traffic_counters": "FETCH_SIZE + WRITE_SIZE per launch, calibrated on a plain copy: bytes between "
                                    "the L2 caches and the fabric, Infinity-Cache hits included (not HBM alone)",
                "algorithmic_bytes_per_launch": bytes_per_su * su_per_launch,
                "bytes_per_su": round(bytes_per_su, 4), "avg_launch_ms": round(avg_s * 1e3, 4),
                "launches": n_l}
    elif not mixed:
        # the lattice stays in LDS for the whole step: bounded by FP32 vector
        # arithmetic (packed FP32 is not used)
        n_l, ms = kt["rs"]
        su_per_launch = su_per_step * args.steps / max(1, n_l)
        avg_s = ms / max(1, n_l) / 1e3
        achieved = FLOPS_PER_SU * su_per_launch / avg_s / 1e12
        roof = {"bound": "alu", "kernel": "resident_step_kernel", "achieved": round(achieved, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": None, "flops_per_su": FLOPS_PER_SU, "avg_launch_ms": round(avg_s * 1e3, 4),
                "launches": n_l}
    else:
        roof = None
    if roof is not None:
        roof["kernel_source_sha256"] = kernel_hash()
        if roof["unit"] == "GB/s":
            roof["measured_copy_GBps"] = copy_rates
            roof["frac_of_hbm_copy"] = round(roof["achieved"] / copy_rates["hbm_1GiB"], 4)

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
            "workload": f"{args.preset}: L={sorted(set(Ls))}, {len(Ls)} samples, {n_chains} chains, "
                        + ("bimodal couplings (D = 0.5, one byte per bond); step" if bimodal
                           else "Gaussian 3x3 couplings; step") + f" = {n_hb} HB + "
                        + ("L" if n_or == ptsg.PT_OR_L else str(n_or)) + " OR sweeps + PT pass"
                        + (f", measurement ({'+'.join(p.get('measure', ('overlap', 'chiral', 'sd')))}) "
                           f"every {every} steps" if every else ""),
            "L": L if not mixed else sorted(set(Ls)), "samples": len(Ls),
            "temperatures": len(temps[0]) if not mixed else sorted({len(t) for t in temps}),
            "replicas": R, "spin_updates_per_step": su_per_step,
            "mapping": (mapping + " lanes" if not mixed else
                        {str(Lv): maps[Ls.index(Lv)] + " lanes" for Lv in sorted(set(Ls))}),
            "mapping_choice": args.mapping,
            "overrelaxation_order": args.or_order,
            "graphs": not args.no_graphs and not args.persistent,
            "step_launch": "persistent" if args.persistent else "multi-launch",
        },
        "roofline": roof,
    }
    if kt is not None and kt["hb"][0]:
        result["heatbath_avg_launch_ms"] = round(kt["hb"][1] / kt["hb"][0], 4)
    if kt is not None:
        # device time of the sweep kernels alone (no swap, energy finalise,
        # measurement or launch gaps), per spin update
        sweep_ms = kt["or"][1] + kt["hb"][1] + kt["rs"][1] + kt["ps"][1]
        result["sweep_kernels_ps_per_su"] = round(sweep_ms * 1e-3 / (args.steps * su_per_step) * 1e12, 4)

    if not args.persistent and not args.no_persistent and not rows:
        # the same workload as one persistent launch per step
        pf = (flags & ~(ptsg.PT_F_RESIDENT | ptsg.PT_F_AUTOTUNE | ptsg.PT_F_GRAPHS)) | ptsg.PT_F_PERSISTENT
        w, su, _, m = run(ptsg, torch, Ls, cpl, temps, R, seed, pf, n_hb, n_or, every, args.steps, 1,
                          timing=False, what=what)
        ps = w / (args.steps * su) * 1e12
        result["persistent_step"] = {"value": round(ps, 4), "unit": "ps/SU", "mapping": m[0] + " lanes",
                                     "ratio_to_value": round(ps / ps_per_su, 3),
                                     "form": "one cooperative launch per step (PT_F_PERSISTENT)"}
    if mixed:
        # each L alone in its own context (per-lattice launches) beside the mixed batch
        per_L = {}
        for Lv in sorted(set(Ls)):
            idx = [i for i, x in enumerate(Ls) if x == Lv]
            w, su, _, m = run(ptsg, torch, [Lv] * len(idx), [cpl[i] for i in idx],
                              [temps[i] for i in idx], R, seed, flags, n_hb, n_or, 0,
                              max(2, args.steps), 1, timing=False)
            per_L[str(Lv)] = {"ps_per_su": round(w / (max(2, args.steps) * su) * 1e12, 3),
                              "mapping": m[0] + " lanes"}
        result["per_L_separate_contexts"] = per_L
        # every lattice in its own context (one sample per launch), one step
        # each after one warm-up step: the unbatched reference
        tot_s = tot_su = 0.0
        for i in range(len(Ls)):
            w, su, _, _ = run(ptsg, torch, [Ls[i]], [cpl[i]], [temps[i]], R, seed, flags & ~ptsg.PT_F_AUTOTUNE,
                              n_hb, n_or, 0, 1, 1, timing=False)
            tot_s += w
            tot_su += su
        per_lattice = tot_s / tot_su * 1e12
        result["one_lattice_per_context"] = {"value": round(per_lattice, 3), "unit": "ps/SU",
                                             "speedup_of_value": round(per_lattice / ps_per_su, 3)}
    elif not args.no_plain and not rows:   # the plain form is checkerboard only
        pflags = ptsg.PT_F_PLAIN | (0 if args.no_graphs else ptsg.PT_F_GRAPHS) | (ptsg.PT_F_BIMODAL if bimodal else 0)
        w, su, _, _ = run(ptsg, torch, Ls, cpl, temps, R, seed, pflags, n_hb, n_or, every, 1, 1,
                          timing=False, what=what)
        plain = w / su * 1e12
        result["plain_single_chain"] = {"value": round(plain, 3), "unit": "ps/SU",
                                        "speedup_of_value": round(plain / ps_per_su, 3),
                                        "form": "site lanes, one chain per workgroup (couplings "
                                                "re-read by every chain), same step"}
    if not args.no_cpu_baseline and not mixed:
        result["cpu_baseline"] = cpu_baseline(L, cpl[0], temps[0], seed, n_hb, n_or)
    elif not args.no_cpu_baseline:
        result["cpu_baseline"] = mixed_cpu_baseline(Ls, cpl, temps, R, seed, n_hb, n_or, ptsg.PT_OR_L)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
