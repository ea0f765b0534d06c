"""Pins of the oracle's lattice, Hamiltonian and local field (Sec. II.A,
Eq. (1); appendix A.1).

- neighbours against coordinates recomputed here;
- the field against the exact gradient -dH/ds taken by automatic
  differentiation of a bond-list energy (catches a transposed backward bond
  or a wrong neighbour);
- the energy against closed forms: a single bond, the aligned ferromagnet
  (appendix A.4 cross-check), time reversal, rotation invariance of the
  isotropic limit (Sec. II.A), and the identity E = -sum over odd sites of
  s.h (every bond has exactly one odd end when L is even).
"""
import numpy as np
import pytest
import torch


def _rand_state(L, rng):
    N = L ** 3
    s = rng.standard_normal((N, 3))
    return s / np.linalg.norm(s, axis=1)[:, None]


@pytest.mark.parametrize("L", [4, 6])
def test_neighbours_brute_force(orc, L):
    for i in range(L ** 3):
        x, y, z = i % L, (i // L) % L, i // (L * L)
        for mu in range(3):
            for d in (+1, -1):
                c = [x, y, z]
                c[mu] = (c[mu] + d) % L
                assert orc.neighbour(L, i, mu, d) == c[0] + L * (c[1] + L * c[2])


def _energy_torch(L, M, s):
    """Bond-list Hamiltonian built from an explicit coordinate list."""
    N = L ** 3
    idx = np.arange(N)
    x, y, z = idx % L, (idx // L) % L, idx // (L * L)
    E = 0.0
    for mu in range(3):
        c = [x.copy(), y.copy(), z.copy()]
        c[mu] = (c[mu] + 1) % L
        j = c[0] + L * (c[1] + L * c[2])
        E = E - torch.einsum("ia,iab,ib->", s, M[mu], s[j])
    return E


@pytest.mark.parametrize("L,seed", [(4, 1), (6, 2)])
def test_field_is_minus_energy_gradient(orc, L, seed):
    rng = np.random.default_rng(seed)
    N = L ** 3
    M = rng.standard_normal((3, N, 3, 3))  # general, non-symmetric bonds
    s = _rand_state(L, rng)
    st = torch.tensor(s, dtype=torch.float64, requires_grad=True)
    E = _energy_torch(L, torch.tensor(M), st)
    (g,) = torch.autograd.grad(E, st)
    h = orc.local_fields(L, M, s)
    np.testing.assert_allclose(h, -g.numpy(), rtol=0, atol=1e-12)
    assert abs(orc.energy(L, M, s) - E.item()) < 1e-11 * N


def test_single_bond_orientation(orc):
    """E = -s_i^T M s_{i+e_mu}: the row index belongs to the first end."""
    L, N = 4, 64
    for mu in range(3):
        M = np.zeros((3, N, 3, 3))
        i = 21
        j = orc.neighbour(L, i, mu, +1)
        M[mu, i, 0, 1] = 1.0
        s = np.zeros((N, 3)); s[:, 2] = 1.0
        s[i] = [1, 0, 0]; s[j] = [0, 1, 0]
        assert orc.energy(L, M, s) == -1.0
        s[i] = [0, 1, 0]; s[j] = [1, 0, 0]
        assert orc.energy(L, M, s) == 0.0
        # field on each end: M s_j at i, M^T s_i at j
        s[i] = [1, 0, 0]; s[j] = [0, 1, 0]
        np.testing.assert_array_equal(orc.local_field(L, M, s, i), [1, 0, 0])
        np.testing.assert_array_equal(orc.local_field(L, M, s, j), [0, 1, 0])


@pytest.mark.parametrize("L", [4, 8])
def test_ferromagnet_ground_state(orc, L):
    N = L ** 3
    M = np.broadcast_to(np.eye(3), (3, N, 3, 3)).copy()
    v = np.array([0.6, 0.0, 0.8])
    s = np.tile(v, (N, 1))
    assert orc.energy(L, M, s) == -3.0 * N
    h = orc.local_field(L, M, s, 5)
    np.testing.assert_allclose(h, 6 * v, atol=1e-15)


def test_time_reversal_and_two_formulas(orc):
    L = 6
    rng = np.random.default_rng(3)
    M = rng.standard_normal((3, L ** 3, 3, 3))
    s = _rand_state(L, rng)
    E = orc.energy(L, M, s)
    assert abs(orc.energy(L, M, -s) - E) < 1e-12
    h = orc.local_fields(L, M, s)
    idx = np.arange(L ** 3)
    odd = ((idx % L + (idx // L) % L + idx // (L * L)) % 2) == 1
    assert abs(-(s[odd] * h[odd]).sum() - E) < 1e-11
    assert abs(-0.5 * (s * h).sum() - E) < 1e-11


def test_isotropic_limit_rotation_invariance(orc):
    """M = J * identity (D = 0): the O(3) symmetry of Sec. II.A."""
    L = 4
    N = L ** 3
    rng = np.random.default_rng(4)
    J = rng.standard_normal((3, N))
    M = J[:, :, None, None] * np.eye(3)
    s = _rand_state(L, rng)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    E0 = orc.energy(L, M, s)
    E1 = orc.energy(L, M, s @ q.T)
    assert abs(E0 - E1) < 1e-12


def test_isotropic_field_matches_scalar_routine(orc):
    """The 3x3 field with M = J * 1 equals the scalar-J Heisenberg field
    h_i = sum_j J_ij s_j, written here from the neighbour list."""
    L = 4
    N = L ** 3
    rng = np.random.default_rng(5)
    J = rng.standard_normal((3, N))
    M = J[:, :, None, None] * np.eye(3)
    s = _rand_state(L, rng)
    h_oracle = orc.local_fields(L, M, s)
    h_scalar = np.zeros((N, 3))
    for i in range(N):
        x, y, z = i % L, (i // L) % L, i // (L * L)
        for mu in range(3):
            cp = [x, y, z]; cp[mu] = (cp[mu] + 1) % L
            cm = [x, y, z]; cm[mu] = (cm[mu] - 1) % L
            jp = cp[0] + L * (cp[1] + L * cp[2])
            jm = cm[0] + L * (cm[1] + L * cm[2])
            h_scalar[i] += J[mu, i] * s[jp] + J[mu, jm] * s[jm]
    np.testing.assert_allclose(h_oracle, h_scalar, rtol=0, atol=1e-14)
