"""Appendix A.4's ferromagnet cross-check on the GPU, in every mapping:
with M = 1 on every bond the aligned state has E = -3N exactly, and after
heat-bath, overrelaxation and tempering the energies the library reports
agree with the FP64 oracle's energy of the same spins to the 7th
significant digit.  The physics is checked too: ordered at T = 0.5 (the
3d Heisenberg ferromagnet orders near T = 1.44), disordered at T = 2.5."""
import numpy as np
import pytest

import oracle as O
from paper_1309_1599_amd import ptsg

pytestmark = pytest.mark.gpu

MAPPINGS = {"site": ptsg.PT_F_SITE_LANES, "chain": ptsg.PT_F_CHAIN_LANES, "resident": ptsg.PT_F_RESIDENT}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    ptsg.load_library()


@pytest.mark.parametrize("mapping", MAPPINGS)
def test_ferromagnet_energies(mapping):
    L, R, seed = 8, 2, 616
    N = L ** 3
    temps = [0.5, 1.0, 1.4, 2.5]
    M = np.broadcast_to(np.eye(3, dtype=np.float32), (3, N, 3, 3)).copy()
    ctx = ptsg.pt_init_batch([L], [M], [temps], R, seed, flags=MAPPINGS[mapping])
    up = np.tile(np.array([0.0, 0.0, 1.0], np.float32), (N, 1))
    for r in range(R):
        for k in range(len(temps)):
            ptsg.pt_set_spins(ctx, 0, r, k, up)
    assert np.all(ptsg.pt_get_energy(ctx)[0] == -3.0 * N)
    for _ in range(30):
        ptsg.pt_step(ctx, 1, L)
        ptsg.pt_swap(ctx)
    E = ptsg.pt_get_energy(ctx)[0]                      # (replica, slot)
    M64 = M.astype(np.float64)
    for r in range(R):
        for k in range(len(temps)):
            s = ptsg.pt_get_spins(ctx, 0, r, k).astype(np.float64)
            e_cpu = O.energy(L, M64, s)
            assert abs(E[r, k] - e_cpu) <= 5e-7 * abs(e_cpu), (r, k, E[r, k], e_cpu)
    e = E.mean(axis=0) / N
    assert e[0] < -2.2 and e[-1] > -1.5 and np.all(np.diff(e) > 0), e
    ptsg.pt_free(ctx)
