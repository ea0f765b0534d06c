"""The persistent step (PT_F_PERSISTENT): every half-sweep of a step, over
every sample and L class, in one cooperative launch with grid-wide barriers
between dependent half-sweeps (App. A.3: the lattices of the batch updated
by one program).

The launch runs the same per-workgroup code on the same grid as the
multi-launch path, so the spins, energies and tempering decisions must be
identical bit for bit to those of the multi-launch path with the same
mapping and tile shape; sweeps replayed on the FP64 oracle must match to the
replay rule; the heat-bath counter must advance once per step; and the
mappings the persistent kernel does not cover must be refused."""
import numpy as np
import pytest

import oracle as O
from gpu_helpers import assert_resynced_sweep, energy_scale
from paper_1309_1599_amd import inputs, ptsg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    ptsg.load_library()


# (name, L per sample, temperatures per sample, replicas, mapping flag, n_or)
CASES = [
    # two samples of 64 chains each: chain lanes chosen automatically
    ("chain", [24, 24], [32, 32], 2, 0, 3),
    # 70 chains: a full group and a ragged one, rows split unevenly
    ("chain-ragged", [20], [35], 2, ptsg.PT_F_CHAIN_LANES, 2),
    # site lanes with several chains per workgroup, two L
    ("site", [12, 12, 8], [5, 5, 3], 3, 0, 2),
    # an uneven batch under the paper's step (1 HB + L OR per sample)
    ("mixed", [8, 12, 16, 24], [4, 5, 6, 8], 2, 0, ptsg.PT_OR_L),
    # one-byte bimodal couplings (site lanes, and chain lanes)
    ("bimodal", [8, 12], [4, 4], 2, ptsg.PT_F_BIMODAL, 2),
    ("chain-bimodal", [24], [32], 2, ptsg.PT_F_BIMODAL, 2),
]


def _inputs(Ls, Ts, seed, bimodal):
    temps = [inputs.geometric_temps(0.6, 1.6, T) for T in Ts]
    if bimodal:
        cpl = [inputs.bimodal_couplings(L, 0.5, seed, s) for s, L in enumerate(Ls)]
    else:
        cpl = [inputs.gaussian_couplings(L, seed, s) for s, L in enumerate(Ls)]
    return temps, cpl


def _state(ctx, Ls, Ts, R):
    spins = [ptsg.pt_get_spins(ctx, s, r, k) for s in range(len(Ls)) for r in range(R) for k in range(Ts[s])]
    perms = [ptsg.pt_get_perm(ctx, s, r) for s in range(len(Ls)) for r in range(R)]
    return spins, perms, ptsg.pt_get_energy(ctx), ptsg.pt_get_counters(ctx)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_persistent_bit_identical_to_launches(case):
    name, Ls, Ts, R, flag, n_or = case
    seed = 5100 + sum(Ls)
    temps, cpl = _inputs(Ls, Ts, seed, flag & ptsg.PT_F_BIMODAL)
    per = ptsg.pt_init_batch(Ls, cpl, temps, R, seed, flags=flag | ptsg.PT_F_PERSISTENT)
    maps = {ptsg.pt_get_mapping(per, s) for s in range(len(Ls))}
    assert len(maps) == 1 and maps <= {ptsg.PT_F_SITE_LANES, ptsg.PT_F_CHAIN_LANES}, maps
    mapping = maps.pop()
    if name.startswith("chain"):
        assert mapping == ptsg.PT_F_CHAIN_LANES
    else:
        assert mapping == ptsg.PT_F_SITE_LANES
    multi = ptsg.pt_init_batch(Ls, cpl, temps, R, seed,
                               flags=(flag & ptsg.PT_F_BIMODAL) | mapping | ptsg.PT_F_GRAPHS)
    for s in range(len(Ls)):
        assert ptsg.pt_get_tile(per, s) == ptsg.pt_get_tile(multi, s)
    for _ in range(3):
        for ctx in (per, multi):
            ptsg.pt_step(ctx, 1, n_or)
            ptsg.pt_swap(ctx)
    a, b = _state(per, Ls, Ts, R), _state(multi, Ls, Ts, R)
    for x, y in zip(a[0], b[0]):
        np.testing.assert_array_equal(x, y, err_msg=f"{name}: spins")
    for x, y in zip(a[1], b[1]):
        np.testing.assert_array_equal(x, y, err_msg=f"{name}: permutations")
    for x, y in zip(a[2], b[2]):
        np.testing.assert_array_equal(x, y, err_msg=f"{name}: energies")
    assert a[3] == b[3] == (3, 3)
    ptsg.pt_free(per)
    ptsg.pt_free(multi)


@pytest.mark.parametrize("L,T,R,flag", [(8, 3, 2, 0), (24, 32, 2, ptsg.PT_F_CHAIN_LANES)],
                         ids=["site-L8", "chain-L24"])
def test_persistent_sweeps_match_oracle(L, T, R, flag):
    """One overrelaxation step, then one heat-bath step, each checked site
    by site on the oracle (re-synced between the two half-sweeps) from the
    state the GPU started from; the chain-lane case on a few chains,
    including the last of the group.  Energies against the oracle's energy
    of the GPU's spins."""
    seed = 5300 + L
    temps = inputs.geometric_temps(0.6, 1.6, T)
    cpl = [inputs.gaussian_couplings(L, seed)]
    ctx = ptsg.pt_init_batch([L], cpl, [temps], R, seed, flags=flag | ptsg.PT_F_PERSISTENT)
    M = cpl[0].astype(np.float64)
    chains = [(r, k) for r in range(R) for k in range(T)]
    if len(chains) > 6:
        chains = [chains[0], chains[1], chains[T - 1], chains[-2], chains[-1]]
    for r in range(R):
        for k in range(T):
            ptsg.pt_set_spins(ctx, 0, r, k, inputs.random_spins(L ** 3, seed, 0, r, k))
    for kind, n_hb, n_or in ((0, 0, 1), (1, 1, 0)):
        start = {key: ptsg.pt_get_spins(ctx, 0, *key) for key in chains}
        ptsg.pt_step(ctx, n_hb, n_or)
        E = ptsg.pt_get_energy(ctx)[0]
        for (r, k) in chains:
            after = ptsg.pt_get_spins(ctx, 0, r, k)
            assert_resynced_sweep(L, M, start[(r, k)], after, kind, 1.0 / temps[k], seed, 0, 0, k, r,
                                  what=f"persistent kind={kind} r={r} k={k}")
            assert abs(E[r, k] - O.energy(L, M, after.astype(np.float64))) <= \
                1e-6 * energy_scale(L, M, after), (kind, r, k)
    assert ptsg.pt_get_counters(ctx) == (1, 0)
    ptsg.pt_free(ctx)


def test_persistent_one_launch_per_step():
    Ls, Ts, R, seed = [8, 12], [4, 4], 2, 5500
    temps, cpl = _inputs(Ls, Ts, seed, False)
    ctx = ptsg.pt_init_batch(Ls, cpl, temps, R, seed, flags=ptsg.PT_F_PERSISTENT)
    ptsg.pt_profile(ctx, True)
    for _ in range(3):
        ptsg.pt_step(ctx, 2, ptsg.PT_OR_L)
    n, ms = ptsg.pt_kernel_time(ctx, ptsg.PT_K_PERSISTENT)
    assert n == 3 and ms > 0.0
    for kind in (ptsg.PT_K_OVERRELAX, ptsg.PT_K_HEATBATH, ptsg.PT_K_RESIDENT):
        assert ptsg.pt_kernel_time(ctx, kind)[0] == 0
    assert ptsg.pt_get_counters(ctx) == (6, 0)
    ptsg.pt_free(ctx)


def test_persistent_refuses_uncovered_mappings():
    L, seed = 8, 5600
    cpl = [inputs.gaussian_couplings(L, seed)]
    temps = [inputs.geometric_temps(0.6, 1.6, 2)]
    for extra in (ptsg.PT_F_RESIDENT, ptsg.PT_F_ROW_OR):
        with pytest.raises(ptsg.PtError) as e:
            ptsg.pt_init_batch([L], cpl, temps, 2, seed, flags=ptsg.PT_F_PERSISTENT | extra)
        assert e.value.status == ptsg.PT_EINVAL


def test_persistent_mapping_rule():
    """One mapping for the whole batch: chain lanes only when they pay for
    every sample (or are forced), else site lanes."""
    seed = 5700

    def mapping(Ls, Ts, R, flag=0):
        temps, cpl = _inputs(Ls, Ts, seed, False)
        ctx = ptsg.pt_init_batch(Ls, cpl, temps, R, seed, flags=flag | ptsg.PT_F_PERSISTENT)
        m = [ptsg.pt_get_mapping(ctx, s) for s in range(len(Ls))]
        ptsg.pt_free(ctx)
        return m

    assert mapping([24], [32], 2) == [ptsg.PT_F_CHAIN_LANES]
    assert mapping([24, 12], [32, 32], 2) == [ptsg.PT_F_SITE_LANES] * 2
    assert mapping([24], [20], 2) == [ptsg.PT_F_SITE_LANES]           # 40 of 64 lanes
    assert mapping([12], [4], 2, ptsg.PT_F_CHAIN_LANES) == [ptsg.PT_F_CHAIN_LANES]
    assert mapping([24], [32], 2, ptsg.PT_F_SITE_LANES) == [ptsg.PT_F_SITE_LANES]
