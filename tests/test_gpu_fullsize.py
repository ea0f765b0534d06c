"""Parity at the presets' full sizes and in the launch configuration the
library picks for them, on sampled outputs the oracle computes one by one:

- L64x8: L = 64, 8 samples x 32 temperatures x 4 replicas (chain lanes);
- L32x64: L = 32, 64 samples x 24 temperatures x 4 replicas (site lanes,
  96 chains per workgroup: the software-pipelined chain loop at its full
  length);
- mixedL: L in {8, 12, 16, 24, 32, 48}, 16 samples each (resident lattices
  up to L = 16, site lanes with 6 and 28 chains per workgroup at L = 24 and
  32, chain lanes at L = 48), with the automatic mappings and with the
  autotuner's.

Within a half-sweep every site of the active colour is updated from its
neighbours of the other colour only, so a site's new value is a function of
(pre-sweep state of the other colour, its own old value).  For colour-0
sites the neighbours are the pre-sweep state; for colour-1 sites they are
the post-sweep colour-0 values.  The oracle recomputes sampled sites from
exactly those inputs, which checks the kernel without any trajectory
divergence.  The sampled chains include the first and last chain of a
workgroup and both sides of a workgroup boundary.  Energies, the tempering
pass and measurement records are checked on whole chains.
"""
import numpy as np
import pytest

import oracle as O
from gpu_helpers import TOL, H_C, colours, energy_scale
from paper_1309_1599_amd import inputs, ptsg

pytestmark = pytest.mark.gpu

N_SITES = 1500


def _chains_of(name, Ls, temps, R):
    """Sampled (sample, replica, slot) triples.  Before the first swap chain
    (r, j) sits at slot j, so local chain index r*T + k names the workgroup
    position."""
    if name == "L64x8":
        return [(0, 0, 0), (3, 2, 17), (7, 3, 31)]
    if name == "L32x64":
        # 96 chains per workgroup: first, second, middle and last chain
        return [(0, 0, 0), (0, 0, 1), (31, 2, 0), (63, 3, 23)]
    out = []
    for L in sorted(set(Ls)):
        s0 = Ls.index(L)
        T = len(temps[s0])
        last = len(Ls) - 1 - Ls[::-1].index(L)
        # local chains 5/6 and 27/28 straddle the 6- and 28-chain workgroups
        # of L = 24 and 32; the last chain of the last sample of every class
        for j in (5, 6, 27, 28):
            if j < R * T and (L in (24, 32)):
                out.append((s0, j // T, j % T))
        out.append((last, R - 1, T - 1))
        out.append((s0, 0, 0))
    return out


PRESETS = [("L64x8", 0), ("L32x64", 0), ("mixedL", 0), ("mixedL", ptsg.PT_F_AUTOTUNE)]


@pytest.fixture(scope="module", params=PRESETS, ids=["L64x8", "L32x64", "mixedL", "mixedL-autotune"])
def big(request):
    import torch
    assert torch.cuda.is_available()
    name, flags = request.param
    Ls, cpl, temps, R, seed = inputs.preset_inputs(name)
    print(f"[fullsize] preset {name} flags {flags}", flush=True)
    ctx = ptsg.pt_init_batch(Ls, cpl, temps, R, seed, flags=flags)
    maps = {L: ptsg.pt_get_mapping(ctx, Ls.index(L)) for L in sorted(set(Ls))}
    print(f"[fullsize] mappings by L: {maps}", flush=True)
    yield dict(ctx=ctx, Ls=Ls, cpl=cpl, temps=temps, R=R, seed=seed, name=name,
               chains=_chains_of(name, Ls, temps, R))
    ptsg.pt_free(ctx)


def _check_sweep(b, kind):
    ctx = b["ctx"]
    rng = np.random.default_rng(5 + kind)
    hb = ptsg.pt_get_counters(ctx)[0]
    before = {c: ptsg.pt_get_spins(ctx, *c) for c in b["chains"]}
    ptsg.pt_step(ctx, 1 if kind == 1 else 0, 0 if kind == 1 else 1)
    E = ptsg.pt_get_energy(ctx)
    key = [b["seed"] & 0xFFFFFFFF, b["seed"] >> 32]
    worst = 0.0
    for (s, r, k) in b["chains"]:
        L = b["Ls"][s]
        N = L ** 3
        col = colours(L)
        M = b["cpl"][s].astype(np.float64)
        after = ptsg.pt_get_spins(ctx, s, r, k)
        mixed = np.where(col[:, None] == 0, after, before[(s, r, k)]).astype(np.float64)
        pre0 = before[(s, r, k)].astype(np.float64)
        beta = 1.0 / b["temps"][s][k]
        sites = list(rng.choice(N, min(N, N_SITES), replace=False)) + [0, N - 1]
        for i in sites:
            state = pre0 if col[i] == 0 else mixed
            h = O.local_field(L, M, state, int(i))
            if kind == 0:
                ref = O.overrelax_spin(h, state[i])
            else:
                w = O.philox(key, [int(i), hb, s, O.ctr3(O.TAG_HB, k, r)])
                ref = O.heatbath_spin(h, beta, O.u23(w[0]), O.u23(w[1]))
            d = np.linalg.norm(after[i] - ref)
            bound = TOL * max(1.0, H_C / np.linalg.norm(h))
            assert d <= bound, (kind, s, r, k, int(i), d, np.linalg.norm(h))
            worst = max(worst, d)
        Eref = O.energy(L, M, after.astype(np.float64))
        assert abs(E[s][r, k] - Eref) <= 1e-6 * energy_scale(L, M, after), (s, r, k)
    return worst


def test_fullsize_heatbath_sweep(big):
    _check_sweep(big, 1)


def test_fullsize_overrelaxation_sweep(big):
    _check_sweep(big, 0)


def test_fullsize_tempering(big):
    ctx = big["ctx"]
    E = ptsg.pt_get_energy(ctx)
    R = big["R"]
    perms = {(s, r): ptsg.pt_get_perm(ctx, s, r) for s in range(ctx.n_samples) for r in range(R)}
    p = ptsg.pt_get_counters(ctx)[1]
    ptsg.pt_swap(ctx)
    for (s, r), perm in perms.items():
        T = len(perm)
        Ech = np.empty(T)
        Ech[perm] = E[s][r]
        ref = perm.copy()
        O.pt_pass(1.0 / big["temps"][s], Ech, ref, big["seed"], p, s, r)
        np.testing.assert_array_equal(ptsg.pt_get_perm(ctx, s, r), ref, err_msg=f"{s},{r}")


def test_fullsize_measure_sampled_records(big):
    ctx = big["ctx"]
    recs = ptsg.pt_measure(ctx, ptsg.PT_M_ALL)
    assert len(recs) == ctx.n_records
    for n in sorted({0, len(recs) // 3, len(recs) // 2 + 5, len(recs) - 1}):
        g = recs[n]
        s, k, a, bb = int(g["sample"]), int(g["tslot"]), int(g["rep_a"]), int(g["rep_b"])
        L = big["Ls"][s]
        sa = ptsg.pt_get_spins(ctx, s, a, k).astype(np.float64)
        sb = ptsg.pt_get_spins(ctx, s, bb, k).astype(np.float64)
        ref = O.overlaps(L, sa, sb)
        for key in ("q0", "qk_re", "qk_im", "cg0", "cgk_re", "cgk_im"):
            np.testing.assert_allclose(g[key], ref[key], rtol=0, atol=1e-12, err_msg=key)
        M = big["cpl"][s].astype(np.float64)
        sd1, sd2 = O.sd_sums(L, M, sa)
        assert abs(g["sd1_a"] - sd1) <= 1e-12 * abs(sd1) and abs(g["sd2_a"] - sd2) <= 1e-12 * abs(sd2)


@pytest.mark.parametrize("L,flags", [(128, 0), (128, ptsg.PT_F_CHAIN_LANES), (256, 0)],
                         ids=["128-site", "128-chain", "256-site"])
def test_largest_lattice_single_chain(L, flags):
    """L = 128 (N = 2^21) in both sweep mappings and L = 256 (N = 2^24, the
    largest size the library accepts): indexing beyond the presets' range,
    sampled sites of one overrelaxation sweep, corners and faces of the
    periodic box included."""
    seed = 901
    cpl = inputs.gaussian_couplings(L, seed)
    ctx = ptsg.pt_init_batch([L], [cpl], [[1.0]], 1, seed, flags=flags)
    before = ptsg.pt_get_spins(ctx, 0, 0, 0)
    ptsg.pt_step(ctx, 0, 1)
    after = ptsg.pt_get_spins(ctx, 0, 0, 0)
    col = colours(L)
    M = cpl.astype(np.float64)
    mixed = np.where(col[:, None] == 0, after, before).astype(np.float64)
    rng = np.random.default_rng(3)
    # include the corners and faces of the periodic box
    sites = list(rng.choice(L ** 3, 800, replace=False)) + [0, L - 1, L * L - 1, L ** 3 - 1]
    for i in sites:
        state = before.astype(np.float64) if col[i] == 0 else mixed
        h = O.local_field(L, M, state, int(i))
        ref = O.overrelax_spin(h, state[i])
        assert np.linalg.norm(after[i] - ref) <= TOL * max(1.0, H_C / np.linalg.norm(h))
    ptsg.pt_free(ctx)
