"""Degenerate inputs on the GPU, through the C ABI, in every mapping:
all couplings zero (|h| = 0 everywhere: overrelaxation must leave every spin
as it is, heat-bath must draw the uniform law from the same counters as the
oracle, the energy is exactly 0), a single temperature with a single
replica (tempering has nothing to exchange, there are no replica pairs),
and the smallest lattice, L = 4, where all mappings must agree bit for bit."""
import numpy as np
import pytest

from gpu_helpers import assert_spins_close, replay_sweep
from paper_1309_1599_amd import inputs, ptsg

pytestmark = pytest.mark.gpu

MAPPINGS = {"site": ptsg.PT_F_SITE_LANES, "chain": ptsg.PT_F_CHAIN_LANES, "resident": ptsg.PT_F_RESIDENT}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    ptsg.load_library()


@pytest.mark.parametrize("mapping", MAPPINGS)
def test_zero_couplings(mapping):
    L, T, R, seed = 8, 2, 2, 404
    temps = [0.7, 1.3]
    M = np.zeros((3, L ** 3, 3, 3), np.float32)
    ctx = ptsg.pt_init_batch([L], [M], [temps], R, seed, flags=MAPPINGS[mapping])
    s0 = {(r, k): ptsg.pt_get_spins(ctx, 0, r, k) for r in range(R) for k in range(T)}
    assert np.all(ptsg.pt_get_energy(ctx)[0] == 0.0)
    ptsg.pt_step(ctx, 0, 3)                       # overrelaxation: no move at h = 0
    for key, s in s0.items():
        np.testing.assert_array_equal(ptsg.pt_get_spins(ctx, 0, *key), s)
    ptsg.pt_step(ctx, 1, 0)                       # heat-bath: uniform draws, same counters as the oracle
    for (r, k), s in s0.items():
        ref, hmag = replay_sweep(L, M.astype(np.float64), s, 1, 1.0 / temps[k], seed, 0, 0, k, r)
        got = ptsg.pt_get_spins(ctx, 0, r, k)
        assert_spins_close(got, ref, np.full(L ** 3, 1e30), what=f"{mapping} r={r} k={k}")
        assert np.abs(np.linalg.norm(got, axis=1) - 1).max() < 1e-6
    assert np.all(ptsg.pt_get_energy(ctx)[0] == 0.0)
    ptsg.pt_swap(ctx)                             # all energies equal: every swap is accepted
    for r in range(R):
        np.testing.assert_array_equal(ptsg.pt_get_perm(ctx, 0, r), [1, 0])
    ptsg.pt_free(ctx)


@pytest.mark.parametrize("mapping", MAPPINGS)
def test_single_temperature_single_replica(mapping):
    L, seed = 8, 405
    M = inputs.gaussian_couplings(L, seed)
    ctx = ptsg.pt_init_batch([L], [M], [[1.1]], 1, seed, flags=MAPPINGS[mapping])
    for _ in range(3):
        ptsg.pt_step(ctx, 1, 2)
        ptsg.pt_swap(ctx)
    np.testing.assert_array_equal(ptsg.pt_get_perm(ctx, 0, 0), [0])
    assert ptsg.pt_get_counters(ctx) == (3, 3)
    assert len(ptsg.pt_measure(ctx, ptsg.PT_M_SD)) == 0
    with pytest.raises(ptsg.PtError):
        ptsg.pt_measure(ctx, ptsg.PT_M_OVERLAP)
    assert np.isfinite(ptsg.pt_get_energy(ctx)).all()
    ptsg.pt_free(ctx)


def test_smallest_lattice_all_mappings_agree():
    L, T, R, seed = 4, 32, 2, 406                  # 64 chains: one full wave in chain lanes
    temps = [inputs.geometric_temps(0.5, 2.0, T)]
    M = [inputs.gaussian_couplings(L, seed)]
    out = {}
    for name, f in MAPPINGS.items():
        ctx = ptsg.pt_init_batch([L], M, temps, R, seed, flags=f)
        assert ptsg.pt_get_mapping(ctx, 0) == f
        for _ in range(3):
            ptsg.pt_step(ctx, 1, 4)
            ptsg.pt_swap(ctx)
        out[name] = ([ptsg.pt_get_spins(ctx, 0, r, k) for r in range(R) for k in (0, 13, T - 1)],
                     [ptsg.pt_get_perm(ctx, 0, r) for r in range(R)], ptsg.pt_get_energy(ctx))
        ptsg.pt_free(ctx)
    for other in ("chain", "resident"):
        for a, b in zip(out["site"][0], out[other][0]):
            np.testing.assert_array_equal(a, b)
        for a, b in zip(out["site"][1], out[other][1]):
            np.testing.assert_array_equal(a, b)
        np.testing.assert_allclose(out["site"][2], out[other][2], rtol=1e-12, atol=1e-12)


def test_all_perms_in_one_call():
    """pt_get_perms returns what pt_get_perm gives per (sample, replica),
    on a batch whose samples differ in L and in the number of temperatures."""
    Ls, Ts, R, seed = [8, 12, 8], [5, 9, 3], 3, 407
    M = [inputs.gaussian_couplings(L, seed, s) for s, L in enumerate(Ls)]
    temps = [inputs.geometric_temps(0.6, 1.8, T) for T in Ts]
    ctx = ptsg.pt_init_batch(Ls, M, temps, R, seed)
    for _ in range(6):
        ptsg.pt_step(ctx, 1, 2)
        ptsg.pt_swap(ctx)
    allp = ptsg.pt_get_perms(ctx)
    moved = 0
    for s, T in enumerate(Ts):
        assert allp[s].shape == (R, T)
        for r in range(R):
            np.testing.assert_array_equal(allp[s][r], ptsg.pt_get_perm(ctx, s, r))
            assert sorted(allp[s][r].tolist()) == list(range(T))
            moved += int(np.any(allp[s][r] != np.arange(T)))
    assert moved > 0
    ptsg.pt_free(ctx)
