"""CPU pins of the host analysis (paper_1309_1599_amd.analysis).

Records come from the FP64 oracle (its Fourier sums are pinned against
numpy's FFT elsewhere).  Pins: infinite-temperature closed forms of the
susceptibilities, a plane-wave overlap field with a known Fourier
coefficient, the lattice Ornstein-Zernike form that the second-moment
correlation length inverts exactly, jackknife identities, the logarithmic
bins, the autocorrelation time of an AR(1) process, and crossings of
curves with known intersections."""
import numpy as np
import pytest

import oracle as O
from oracle import OracleEnsemble
from paper_1309_1599_amd import analysis as A
from paper_1309_1599_amd import inputs, ptsg


def _random_records(L, n, seed):
    """n independent pairs of hot-start configurations (beta = 0)."""
    out = []
    for m in range(n):
        sa = O.init_spins(L, seed, m, 0, 0)
        sb = O.init_spins(L, seed, m, 0, 1)
        rec = O.overlaps(L, sa, sb)
        rec.update(sample=0, tslot=0, rep_a=0, rep_b=1)
        out.append([rec])
    return A.stack(out)


def test_infinite_temperature_susceptibilities():
    """Independent uniform spins: <(s^a.s^b)^2> = 1/3 and the site terms are
    uncorrelated, so chi_SG(k) = 1/3 at every k; <zeta^2> = 2/9 and the
    chiralities are pairwise uncorrelated, so chi_CG(k) = 4/81; xi = 0."""
    L, n = 4, 600
    R = _random_records(L, n, 77)
    F = A.fields(R, L)
    N = L ** 3
    blocks = {k: F[k][:, 0].reshape(20, -1).mean(axis=1) for k in ("q2", "qk2", "cg2", "cgk2")}
    for key, want in (("q2", 1 / 3), ("qk2", 1 / 3), ("cg2", 4 / 81), ("cgk2", 4 / 81)):
        m, e = A.jackknife(N * blocks[key])
        assert abs(m - want) < 4 * e, (key, m, e, want)
    chi = A.susceptibilities({k: blocks[k].mean() for k in blocks}, L)
    xi, err = A.jackknife(np.stack([N * blocks["q2"], N * blocks["qk2"]], axis=1),
                          lambda m: A.xi_second_moment(m[0], m[1], L))
    assert xi < 4 * err + 0.05
    assert chi["chi_sg0"] == pytest.approx(N * blocks["q2"].mean())


def test_plane_wave_overlap():
    """q_x = cos(2 pi x / L): q(0) = 0 and q(k_x) = 1/2, q(k_y) = q(k_z) = 0,
    so |q(k_min)|^2 averaged over directions is 1/12."""
    L = 6
    N = L ** 3
    x = np.arange(N) % L
    sa = np.tile([0.0, 0.0, 1.0], (N, 1))
    th = 2 * np.pi * x / L
    sb = np.stack([np.sin(th), np.zeros(N), np.cos(th)], axis=1)
    rec = O.overlaps(L, sa, sb)
    rec.update(sample=0, tslot=0, rep_a=0, rep_b=1)
    F = A.fields(A.stack([[rec]]), L)
    assert F["q"][0, 0] == pytest.approx(0.0, abs=1e-14)
    assert F["qk2"][0, 0] == pytest.approx(1 / 12, rel=1e-12)


def test_xi_inverts_lattice_ornstein_zernike():
    """chi(k) = chi0 / (1 + 4 xi^2 sin^2(k/2)) gives back xi exactly."""
    for L in (8, 16, 64):
        for xi in (0.3, 2.0, 11.0):
            chi0 = 5.0
            chik = chi0 / (1 + 4 * xi ** 2 * np.sin(np.pi / L) ** 2)
            assert A.xi_second_moment(chi0, chik, L) == pytest.approx(xi, rel=1e-12)


def test_jackknife_identities():
    rng = np.random.default_rng(3)
    x = rng.normal(size=37)
    m, e = A.jackknife(x)
    assert m == pytest.approx(x.mean())
    assert e == pytest.approx(x.std(ddof=1) / np.sqrt(len(x)), rel=1e-12)
    # a nonlinear function against the delete-one definition written out
    y = rng.normal(2.0, 0.1, size=37)
    b = np.stack([x + 5, y], axis=1)
    m, e = A.jackknife(b, lambda v: v[0] / v[1])
    jk = np.array([np.delete(x + 5, i).mean() / np.delete(y, i).mean() for i in range(37)])
    assert m == pytest.approx((x + 5).mean() / y.mean())
    assert e == pytest.approx(np.sqrt(36 / 37 * ((jk - jk.mean()) ** 2).sum()), rel=1e-10)
    with pytest.raises(ValueError):
        A.jackknife(x[:1])


def test_log_bins_and_thermalisation():
    assert A.log_bins(16) == [(8, 16), (4, 8), (2, 4), (1, 2)]
    assert A.log_bins(100)[0] == (50, 100)
    # a constant series per sample is thermalised at every bin
    flat = np.tile(np.arange(5.0), (64, 1))
    for lo, hi, d, e in A.thermalisation(flat):
        assert d == 0.0 and e == 0.0
    # a relaxing series: <O(i)> - <O(i_f)> is negative and shrinks towards the end
    t = np.arange(1, 1025)[:, None] * np.ones((1, 8))
    res = A.thermalisation(-1.0 / t)
    diffs = [d for _, _, d, _ in res]
    assert diffs[0] == 0.0 and all(a > b for a, b in zip(diffs[1:], diffs[2:]))


def test_tau_int_ar1():
    rng = np.random.default_rng(11)
    for rho in (0.0, 0.8):
        n = 200000
        eps = rng.normal(size=n)
        x = np.empty(n)
        x[0] = eps[0]
        for i in range(1, n):
            x[i] = rho * x[i - 1] + eps[i]
        want = (1 + rho) / (2 * (1 - rho))
        assert A.tau_int(x) == pytest.approx(want, rel=0.1)


def test_crossing_and_nu():
    T = np.linspace(0.5, 1.5, 11)
    y1 = 1 + 2 * (T - 1.0)
    y2 = 1 - (T - 1.0)
    tc, yc, s1, s2 = A.crossing(T, y1, y2)
    assert tc == pytest.approx(1.0) and yc == pytest.approx(1.0)
    assert s1 == pytest.approx(2.0) and s2 == pytest.approx(-1.0)
    q1 = 0.2 + (T - 0.9) ** 2
    q2 = 0.2 + 0.5 * (T - 0.9)
    tc, yc, _, _ = A.crossing(T, q1, q2, order=2)
    assert tc in (pytest.approx(0.9), pytest.approx(1.4))
    with pytest.raises(ValueError):
        A.crossing(T, y1, y1 + 1)
    assert A.nu_from_slope_ratio(2 ** (1 + 1 / 0.8)) == pytest.approx(0.8)
    res = A.crossing_jackknife(T, np.tile(y1, (5, 1)), np.tile(y2, (5, 1)))
    assert res["T_cross"][0] == pytest.approx(1.0) and res["T_cross"][1] == pytest.approx(0.0, abs=1e-12)
    assert res["slope_ratio"][0] == pytest.approx(-0.5)


def test_thermal_means_of_an_oracle_run():
    """Records of an oracle run group by (sample, slot); the energy per spin
    of each slot equals the mean over the run of the chains at that slot."""
    L, T, R = 4, 3, 3
    temps = inputs.linear_temps(0.5, 1.5, T)
    ens = OracleEnsemble(L, inputs.gaussian_couplings(L, 5), temps, R, 9)
    recs, energies = [], []
    for _ in range(6):
        ens.step(1, 2)
        ens.swap()
        recs.append(ens.measure())
        energies.append([[ens.E[r, ens.perm[r, k]] for k in range(T)] for r in range(R)])
    Rr = A.stack(recs)
    assert Rr.shape == (6, T * R * (R - 1) // 2)
    keys, means = A.thermal_means(Rr, L)
    assert keys == [(0, k) for k in range(T)]
    want = np.asarray(energies).mean(axis=(0, 1)) / L ** 3
    np.testing.assert_allclose(means["e"], want, rtol=1e-12)
    assert Rr.dtype == ptsg.MEAS_DTYPE


def test_crossing_extrapolated_just_beyond_the_grid():
    """Lines meeting slightly below the grid: found with extrapolation
    allowed, refused without it or when too far out."""
    T = np.linspace(1.0, 1.4, 9)
    y1 = 0.6 - 0.8 * (T - 0.95)
    y2 = 0.6 - 1.2 * (T - 0.95)
    tc, yc, s1, s2 = A.crossing(T, y1, y2, extrapolate=0.25)
    assert tc == pytest.approx(0.95) and yc == pytest.approx(0.6)
    with pytest.raises(ValueError):
        A.crossing(T, y1, y2)
    with pytest.raises(ValueError):
        A.crossing(T, 0.6 - 0.8 * (T - 0.5), 0.6 - 1.2 * (T - 0.5), extrapolate=0.25)


def test_temperature_walk_tau_two_state():
    """Two temperatures, one replica: the two chains sit in opposite slots and
    trade places with probability p per step.  Each slot series is a two-state
    Markov chain with rho(t) = (1 - 2p)^t, so tau = (1 - p) / (2p)."""
    rng = np.random.default_rng(21)
    for p in (0.5, 0.1):
        n = 400000
        flips = rng.random(n) < p
        perm = np.zeros((n, 2), dtype=np.int32)
        perm[:, 0] = np.cumsum(flips) % 2            # chain at slot 0
        perm[:, 1] = 1 - perm[:, 0]
        slots = A.slot_of_chain(perm)
        np.testing.assert_array_equal(np.take_along_axis(slots, perm, axis=1), np.tile([0, 1], (n, 1)))
        assert A.temperature_walk_tau(slots) == pytest.approx((1 - p) / (2 * p), rel=0.05)


def test_slot_of_chain_inverts():
    rng = np.random.default_rng(5)
    perm = np.stack([rng.permutation(9) for _ in range(6)]).reshape(2, 3, 9)
    inv = A.slot_of_chain(perm)
    for idx in np.ndindex(2, 3):
        for k in range(9):
            assert inv[idx][perm[idx][k]] == k
