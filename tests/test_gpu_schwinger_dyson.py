"""The Schwinger-Dyson identity of appendix A.4 on the GPU's own runs: in
equilibrium, averaged over the lattice, 2T <s.h> - <h^2 - (s.h)^2> = 0 at
every temperature.  The paper uses it to test its random numbers; here it
checks the heat-bath draws (Philox, the inverse CDF, the frame) and the
tempering together, in every mapping, on the Gaussian and the bimodal
couplings.  The same data evaluated at a temperature off by 5 % must fail,
so that the test can see a mistake of that size."""
import numpy as np
import pytest

from paper_1309_1599_amd import inputs, ptsg

pytestmark = pytest.mark.gpu

MAPPINGS = {"site": ptsg.PT_F_SITE_LANES, "chain": ptsg.PT_F_CHAIN_LANES, "resident": ptsg.PT_F_RESIDENT}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    ptsg.load_library()


def _sd_series(mapping, couplings, L=8, S=8, n_warm=200, n_meas=400, seed=515):
    temps = inputs.geometric_temps(0.8, 2.0, 4)
    if couplings == "bimodal":
        M = [inputs.bimodal_couplings(L, 1.0, seed, s) for s in range(S)]
        flags = MAPPINGS[mapping] | ptsg.PT_F_BIMODAL
    else:
        M = [inputs.gaussian_couplings(L, seed, s) for s in range(S)]
        flags = MAPPINGS[mapping]
    ctx = ptsg.pt_init_batch([L] * S, M, [temps] * S, 2, seed, flags=flags | ptsg.PT_F_GRAPHS)
    for _ in range(n_warm):
        ptsg.pt_step(ctx, 1, L)
        ptsg.pt_swap(ctx)
    sd1 = np.zeros((n_meas, S, len(temps), 2))
    sd2 = np.zeros_like(sd1)
    for m in range(n_meas):
        ptsg.pt_step(ctx, 1, L)
        ptsg.pt_swap(ctx)
        rec = ptsg.pt_measure(ctx, ptsg.PT_M_SD)
        s, k = rec["sample"], rec["tslot"]
        sd1[m, s, k, 0], sd1[m, s, k, 1] = rec["sd1_a"], rec["sd1_b"]
        sd2[m, s, k, 0], sd2[m, s, k, 1] = rec["sd2_a"], rec["sd2_b"]
    ptsg.pt_free(ctx)
    return np.asarray(temps), sd1 / L ** 3, sd2 / L ** 3


def _z(T, sd1, sd2, n_blocks=20):
    """Per temperature: the lattice-averaged identity, averaged over time,
    replicas and samples, over its error from time blocks x samples."""
    d = 2 * T[None, None, :, None] * sd1 - sd2             # (time, sample, T, replica)
    d = d.mean(axis=3)
    n = d.shape[0] // n_blocks * n_blocks
    blocks = d[:n].reshape(n_blocks, -1, *d.shape[1:]).mean(axis=1)   # (block, sample, T)
    blocks = blocks.reshape(-1, d.shape[2])
    mean = blocks.mean(axis=0)
    err = blocks.std(axis=0, ddof=1) / np.sqrt(blocks.shape[0])
    return mean / err, mean, err


@pytest.mark.parametrize("mapping", MAPPINGS)
@pytest.mark.parametrize("couplings", ["gaussian", "bimodal"])
def test_schwinger_dyson_identity(mapping, couplings):
    T, sd1, sd2 = _sd_series(mapping, couplings)
    z, mean, err = _z(T, sd1, sd2)
    assert np.all(np.abs(z) < 4), (z, mean, err)
    # the identity is sharp: its error is a small fraction of either term
    assert np.all(err < 0.01 * np.abs(sd2).mean(axis=(0, 1, 3))), (err, np.abs(sd2).mean(axis=(0, 1, 3)))
    # a 5 % error in the temperature would be seen
    z_off, _, _ = _z(T * 1.05, sd1, sd2)
    assert np.all(np.abs(z_off) > 6), z_off
