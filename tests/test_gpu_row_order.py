"""Overrelaxation in the row order (PT_F_ROW_OR) against the FP64 oracle's
row sweep, through the C ABI: one sweep replayed update by update on the
states the GPU saw (each spin depends on the FP32 spins updated before it
in its row, so rounding is carried along the row; the per-update replay
holds each FP32 update to the single-update bound, and the whole sweep is
also compared with a looser bound) for L = 8 (where a
row is a whole x line and wraps onto itself), L = 16 and 32 (two and four
rows along x; an odd number above one is refused), energies of the resulting states, energy
conservation over many sweeps, a captured step replayed against the eager
one, and the flag's validation."""
import numpy as np
import pytest

import oracle as O
from gpu_helpers import TOL, assert_energy_close, assert_spins_close
from paper_1309_1599_amd import inputs, ptsg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    ptsg.load_library()


def _row_order(L):
    for cls in (0, 1):
        for z in range(L):
            for y in range(L):
                for b in range(L // 8):
                    if (b + y + z) % 2 == cls:
                        for x in range(8 * b, 8 * b + 8):
                            yield x + L * (y + L * z)


def _replay_each_update(L, M, s0, gpu):
    """Per-update replay: every site is updated by the oracle from the state
    the GPU saw at that moment (GPU values for the sites updated before it
    in the row order, s0 for the others), so each FP32 update is compared on
    identical inputs.  Returns the oracle's updates and |h| at each."""
    state = np.array(s0, dtype=np.float64, copy=True)
    ref = np.empty_like(state)
    hmag = np.zeros(L ** 3)
    for i in _row_order(L):
        h = O.local_field(L, M, state, i)
        hmag[i] = np.linalg.norm(h)
        ref[i] = O.overrelax_spin(h, state[i])
        state[i] = gpu[i]
    return ref, hmag


@pytest.mark.parametrize("L", [8, 16, 32])
def test_row_sweep_matches_oracle(L):
    T, R, seed = 3, 2, 700 + L
    temps = inputs.geometric_temps(0.6, 1.6, T)
    M = inputs.gaussian_couplings(L, seed)
    ctx = ptsg.pt_init_batch([L], [M], [temps], R, seed, flags=ptsg.PT_F_ROW_OR)
    assert ptsg.pt_get_mapping(ctx, 0) == ptsg.PT_F_CHAIN_LANES
    ptsg.pt_step(ctx, 1, 0)   # leave the hot start: a state with fields of all sizes
    s0 = {(r, k): ptsg.pt_get_spins(ctx, 0, r, k) for r in range(R) for k in range(T)}
    ptsg.pt_step(ctx, 0, 1)
    E = ptsg.pt_get_energy(ctx)[0]
    M64 = M.astype(np.float64)
    worst = drift = 0.0
    for r in range(R):
        for k in range(T):
            got = ptsg.pt_get_spins(ctx, 0, r, k)
            ref, hmag = _replay_each_update(L, M64, s0[(r, k)], got)
            mx, _ = assert_spins_close(got, ref, hmag, what=f"L={L} r={r} k={k}")
            worst = max(worst, mx)
            # end to end against the oracle's own sweep: FP32 rounding carried
            # along the rows, so a looser bound
            whole = np.array(s0[(r, k)], dtype=np.float64, copy=True)
            O.row_sweep(L, M64, whole)
            drift = max(drift, np.abs(got - whole).max())
            assert_energy_close(E[r, k], L, M64, got, what=f"L={L} r={r} k={k}")
    print(f"L={L}: per-update max |ds| {worst:.3g} (bound {TOL} scaled by |h|); "
          f"whole sweep max |ds| {drift:.3g}")
    assert drift < 1e-4
    ptsg.pt_free(ctx)


def test_row_order_conserves_energy_and_differs_from_checkerboard():
    L, T, R, seed = 16, 2, 2, 760
    temps = inputs.geometric_temps(0.6, 1.6, T)
    M = inputs.gaussian_couplings(L, seed)
    rows = ptsg.pt_init_batch([L], [M], [temps], R, seed, flags=ptsg.PT_F_ROW_OR)
    cb = ptsg.pt_init_batch([L], [M], [temps], R, seed, flags=ptsg.PT_F_CHAIN_LANES)
    for ctx in (rows, cb):
        ptsg.pt_step(ctx, 1, 0)
    np.testing.assert_array_equal(ptsg.pt_get_spins(rows, 0, 0, 0), ptsg.pt_get_spins(cb, 0, 0, 0))
    E0 = ptsg.pt_get_energy(rows)[0].copy()
    for ctx in (rows, cb):
        ptsg.pt_step(ctx, 0, 50)
    E1 = ptsg.pt_get_energy(rows)[0]
    assert (np.abs(E1 - E0) <= 50 * 1e-5 * np.abs(E0)).all(), np.abs(E1 / E0 - 1).max()
    s = ptsg.pt_get_spins(rows, 0, 1, 1)
    assert np.abs(np.linalg.norm(s, axis=1) - 1).max() < 1e-6
    assert np.abs(s - ptsg.pt_get_spins(cb, 0, 1, 1)).max() > 1e-2   # another dynamics
    ptsg.pt_free(rows)
    ptsg.pt_free(cb)


def test_row_order_graph_replays_match_eager():
    L, T, R, seed = 32, 3, 2, 780
    temps = [inputs.geometric_temps(0.7, 1.5, T)]
    cpl = [inputs.gaussian_couplings(L, seed)]
    eager = ptsg.pt_init_batch([L], cpl, temps, R, seed, flags=ptsg.PT_F_ROW_OR)
    graph = ptsg.pt_init_batch([L], cpl, temps, R, seed, flags=ptsg.PT_F_ROW_OR | ptsg.PT_F_GRAPHS)
    for _ in range(3):
        for ctx in (eager, graph):
            ptsg.pt_step(ctx, 1, 4)
            ptsg.pt_swap(ctx)
        for r in range(R):
            np.testing.assert_array_equal(ptsg.pt_get_perm(eager, 0, r), ptsg.pt_get_perm(graph, 0, r))
            np.testing.assert_array_equal(ptsg.pt_get_spins(eager, 0, r, 0), ptsg.pt_get_spins(graph, 0, r, 0))
        np.testing.assert_array_equal(ptsg.pt_get_energy(eager)[0], ptsg.pt_get_energy(graph)[0])
    ptsg.pt_free(eager)
    ptsg.pt_free(graph)
