"""pt_run: whole Monte Carlo steps (Sec. III: the sweeps of a step, one
tempering pass, a measurement every few steps), each kind of step captured
once as a hipGraph and replayed.  The results must be those of the separate
calls bit for bit -- spins, permutations, energies, counters and every
measurement record -- over several calls in a row (graph replays with host
reads in between), in every mapping and in the persistent step; the
argument checks must refuse what the header says."""
import numpy as np
import pytest

from paper_1309_1599_amd import inputs, ptsg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    ptsg.load_library()


def _batch(seed):
    # resident (L = 8), site lanes (L = 12), chain lanes (L = 24, 64 chains)
    Ls, Ts, R = [8, 12, 24], [4, 5, 32], 2
    temps = [inputs.geometric_temps(0.6, 1.6, T) for T in Ts]
    cpl = [inputs.gaussian_couplings(L, seed, s) for s, L in enumerate(Ls)]
    return Ls, Ts, R, temps, cpl


def _state(ctx, Ls, Ts, R):
    spins = [ptsg.pt_get_spins(ctx, s, r, k) for s in range(len(Ls)) for r in range(R) for k in range(Ts[s])]
    return spins, ptsg.pt_get_perms(ctx), ptsg.pt_get_energy(ctx), ptsg.pt_get_counters(ctx)


def _same(a, b, what):
    for x, y in zip(a[0], b[0]):
        np.testing.assert_array_equal(x, y, err_msg=f"{what}: spins")
    for x, y in zip(a[1], b[1]):
        np.testing.assert_array_equal(x, y, err_msg=f"{what}: permutations")
    for x, y in zip(a[2], b[2]):
        np.testing.assert_array_equal(x, y, err_msg=f"{what}: energies")
    assert a[3] == b[3], what


@pytest.mark.parametrize("flags", [ptsg.PT_F_GRAPHS, ptsg.PT_F_GRAPHS | ptsg.PT_F_PERSISTENT, 0],
                         ids=["graphs", "persistent", "eager"])
def test_run_equals_separate_calls(flags):
    import torch
    seed = 6100
    Ls, Ts, R, temps, cpl = _batch(seed)
    run = ptsg.pt_init_batch(Ls, cpl, temps, R, seed, flags=flags)
    ref = ptsg.pt_init_batch(Ls, cpl, temps, R, seed, flags=flags & ptsg.PT_F_PERSISTENT)
    n_rec = run.n_records
    what = ptsg.PT_M_OVERLAP | ptsg.PT_M_CHIRAL | ptsg.PT_M_ENERGY
    every, n_hb, n_or = 2, 1, ptsg.PT_OR_L
    buf = torch.zeros(3 * n_rec * ptsg.MEAS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    for call, n_steps in enumerate((6, 5, 2)):
        ptsg.pt_run(run, n_steps, n_hb, n_or, every, what, buf.data_ptr(), 3 * n_rec)
        ptsg.pt_sync(run)
        got = np.frombuffer(buf.cpu().numpy().tobytes(), dtype=ptsg.MEAS_DTYPE)
        want = []
        for t in range(n_steps):
            ptsg.pt_step(ref, n_hb, n_or)
            ptsg.pt_swap(ref)
            if (t + 1) % every == 0:
                want.append(ptsg.pt_measure(ref, what))
        for k, w in enumerate(want):
            assert got[k * n_rec:(k + 1) * n_rec].tobytes() == w.tobytes(), (call, k)
        _same(_state(run, Ls, Ts, R), _state(ref, Ls, Ts, R), f"call {call}")
    ptsg.pt_free(run)
    ptsg.pt_free(ref)


@pytest.mark.parametrize("every", [1, 3])
def test_run_many_short_steps(every):
    """One L = 8 sample (resident): runs of 40, 17 and 3 steps, measuring
    every step or every third, each record and the state equal to the
    separate calls (the device record cursor keeps counting across the
    replays of one call)."""
    import torch
    seed = 6300 + every
    L, T, R = 8, 8, 2
    temps = [inputs.linear_temps(0.5, 2.0, T)]
    cpl = [inputs.gaussian_couplings(L, seed)]
    run = ptsg.pt_init_batch([L], cpl, temps, R, seed, flags=ptsg.PT_F_GRAPHS)
    ref = ptsg.pt_init_batch([L], cpl, temps, R, seed)
    n_rec = run.n_records
    what = ptsg.PT_M_OVERLAP | ptsg.PT_M_ENERGY
    cap = 40 // every * n_rec
    buf = torch.zeros(cap * ptsg.MEAS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    for call, n_steps in enumerate((40, 17, 3)):
        ptsg.pt_run(run, n_steps, 1, L, every, what, buf.data_ptr(), cap)
        ptsg.pt_sync(run)
        got = np.frombuffer(buf.cpu().numpy().tobytes(), dtype=ptsg.MEAS_DTYPE)
        k = 0
        for t in range(n_steps):
            ptsg.pt_step(ref, 1, L)
            ptsg.pt_swap(ref)
            if (t + 1) % every == 0:
                w = ptsg.pt_measure(ref, what)
                assert got[k * n_rec:(k + 1) * n_rec].tobytes() == w.tobytes(), (call, t)
                k += 1
        _same(_state(run, [L], [T], R), _state(ref, [L], [T], R), f"call {call}")
    ptsg.pt_free(run)
    ptsg.pt_free(ref)


def test_run_four_replicas_all_measurements():
    """R = 4 (six records per temperature slot, the slot-wise chirality and
    Schwinger-Dyson kernels) with every measurement bit, inside the replayed
    graphs: records and state equal to the separate calls."""
    import torch
    seed = 6400
    Ls, Ts, R = [8, 12], [4, 3], 4
    temps = [inputs.geometric_temps(0.6, 1.6, T) for T in Ts]
    cpl = [inputs.gaussian_couplings(L, seed, s) for s, L in enumerate(Ls)]
    run = ptsg.pt_init_batch(Ls, cpl, temps, R, seed, flags=ptsg.PT_F_GRAPHS)
    ref = ptsg.pt_init_batch(Ls, cpl, temps, R, seed)
    n_rec = run.n_records
    assert n_rec == 6 * sum(Ts)
    buf = torch.zeros(5 * n_rec * ptsg.MEAS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    ptsg.pt_run(run, 5, 1, ptsg.PT_OR_L, 1, ptsg.PT_M_ALL, buf.data_ptr(), 5 * n_rec)
    ptsg.pt_sync(run)
    got = np.frombuffer(buf.cpu().numpy().tobytes(), dtype=ptsg.MEAS_DTYPE)
    for t in range(5):
        ptsg.pt_step(ref, 1, ptsg.PT_OR_L)
        ptsg.pt_swap(ref)
        w = ptsg.pt_measure(ref, ptsg.PT_M_ALL)
        assert got[t * n_rec:(t + 1) * n_rec].tobytes() == w.tobytes(), t
    _same(_state(run, Ls, Ts, R), _state(ref, Ls, Ts, R), "R = 4")
    ptsg.pt_free(run)
    ptsg.pt_free(ref)


def test_run_argument_checks():
    import torch
    seed = 6200
    Ls, Ts, R, temps, cpl = _batch(seed)
    ctx = ptsg.pt_init_batch(Ls, cpl, temps, R, seed, flags=ptsg.PT_F_GRAPHS)
    n_rec = ctx.n_records
    buf = torch.zeros(n_rec * ptsg.MEAS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")

    def status(*args):
        try:
            ptsg.pt_run(ctx, *args)
        except ptsg.PtError as e:
            return e.status
        return ptsg.PT_OK

    assert status(4, 1, 2, 2, ptsg.PT_M_ALL, buf.data_ptr(), n_rec) == ptsg.PT_ENOMEM   # 2 records sets
    assert status(4, 1, 2, 2, ptsg.PT_M_ALL, 0, 0) == ptsg.PT_EINVAL
    assert status(-1, 1, 2) == ptsg.PT_EINVAL
    assert status(2, -1, 2) == ptsg.PT_EINVAL
    assert status(2, 1, 2, 1, 64, buf.data_ptr(), 2 * n_rec) == ptsg.PT_EINVAL         # unknown bits
    assert ptsg.pt_get_counters(ctx) == (0, 0)                                          # nothing ran
    assert status(0, 1, 2, 1, ptsg.PT_M_ALL, 0, 0) == ptsg.PT_OK                        # no steps
    assert status(3, 1, 2) == ptsg.PT_OK                                                # no measurement
    assert status(1, 1, 2, 2, ptsg.PT_M_ALL, 0, 0) == ptsg.PT_OK                        # 1 // 2 = none
    assert ptsg.pt_get_counters(ctx) == (4, 4)
    ptsg.pt_free(ctx)
