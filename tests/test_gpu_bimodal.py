"""The paper's coupling family stored as one byte per bond (PT_F_BIMODAL):
site-lane samples decode the codes in the sweep kernel, chain-lane samples
read each code's matrix from a per-sample table; the result must be
bit-identical to passing the same matrices as floats, for the batched and
the plain form and both mappings, at D = 0.5 and D = 1, and one sweep must
match the oracle replayed on the same state (the oracle takes the
materialised matrices)."""
import numpy as np
import pytest

from gpu_helpers import assert_spins_close, replay_sweep
from paper_1309_1599_amd import inputs, ptsg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    ptsg.load_library()


def _run(Ls, cpl, temps, R, seed, flags):
    ctx = ptsg.pt_init_batch(Ls, cpl, temps, R, seed, flags=flags)
    for _ in range(3):
        ptsg.pt_step(ctx, 1, 3)
        ptsg.pt_swap(ctx)
    T = len(temps[0])
    out = ([ptsg.pt_get_spins(ctx, s, r, k) for s in range(len(Ls)) for r in range(R) for k in (0, T - 1)],
           [ptsg.pt_get_perm(ctx, s, r) for s in range(len(Ls)) for r in range(R)],
           ptsg.pt_get_energy(ctx), [ptsg.pt_get_mapping(ctx, s) for s in range(len(Ls))])
    ptsg.pt_free(ctx)
    return out


@pytest.mark.parametrize("D", [0.5, 1.0])
@pytest.mark.parametrize("form", [ptsg.PT_F_SITE_LANES, ptsg.PT_F_PLAIN, ptsg.PT_F_CHAIN_LANES, 0],
                         ids=["site", "plain", "chain", "auto"])
def test_bytes_bit_identical_to_floats(D, form):
    Ls, T, R, seed = [12, 8, 20], 5, 2, 515
    cpl = [inputs.bimodal_couplings(L, D, seed, s) for s, L in enumerate(Ls)]
    temps = [inputs.geometric_temps(0.6, 1.6, T)] * len(Ls)
    a = _run(Ls, cpl, temps, R, seed, form)
    b = _run(Ls, cpl, temps, R, seed, form | ptsg.PT_F_BIMODAL)
    assert a[3] == b[3]
    for x, y in zip(a[0], b[0]):
        np.testing.assert_array_equal(x, y)
    for x, y in zip(a[1], b[1]):
        np.testing.assert_array_equal(x, y)
    for x, y in zip(a[2], b[2]):
        np.testing.assert_array_equal(x, y)


def test_bytes_chain_lanes_automatic():
    """Full 64-lane waves at L = 24 take chain lanes on their own; two
    samples with different D."""
    Ls, T, R, seed = [24, 24], 32, 2, 717
    cpl = [inputs.bimodal_couplings(24, D, seed, s) for s, D in enumerate((0.5, 1.0))]
    temps = [inputs.geometric_temps(0.6, 1.6, T)] * 2
    a = _run(Ls, cpl, temps, R, seed, 0)
    b = _run(Ls, cpl, temps, R, seed, ptsg.PT_F_BIMODAL)
    assert a[3] == b[3] == [ptsg.PT_F_CHAIN_LANES] * 2
    for x, y in zip(a[0] + a[1] + list(a[2]), b[0] + b[1] + list(b[2])):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("mapping", [ptsg.PT_F_SITE_LANES, ptsg.PT_F_CHAIN_LANES], ids=["site", "chain"])
@pytest.mark.parametrize("kind", [0, 1], ids=["overrelax", "heatbath"])
def test_bytes_one_sweep_matches_oracle(kind, mapping):
    L, T, R, seed = 8, 3, 2, 616
    M = inputs.bimodal_couplings(L, 0.5, seed)
    temps = inputs.linear_temps(0.7, 1.5, T)
    ctx = ptsg.pt_init_batch([L], [M], [temps], R, seed, flags=mapping | ptsg.PT_F_BIMODAL)
    assert ptsg.pt_get_mapping(ctx, 0) == mapping
    s0 = {(r, k): ptsg.pt_get_spins(ctx, 0, r, k) for r in range(R) for k in range(T)}
    ptsg.pt_step(ctx, 1 if kind else 0, 0 if kind else 1)
    M64 = M.astype(np.float64)
    for r in range(R):
        for k in range(T):
            ref, hmag = replay_sweep(L, M64, s0[(r, k)], kind, 1.0 / temps[k], seed, 0, 0, k, r)
            assert_spins_close(ptsg.pt_get_spins(ctx, 0, r, k), ref, hmag, what=f"r={r} k={k}")
    ptsg.pt_free(ctx)
