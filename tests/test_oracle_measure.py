"""Pins of the oracle's observables (Sec. II.B, appendix A.4).

- Fourier sums at k = 0 and k = (2 pi/L) e_d against numpy's FFT of the
  overlap and chiral-overlap fields;
- the chirality against the 3x3 determinant det[s_{x+e}, s_x, s_{x-e}]
  (numpy.linalg.det), which equals the triple product;
- closed forms for independent uniform spins (beta = 0): <q_x^2> = 1/3,
  sum_ab <(s^a_alpha s^b_beta)^2> = 1, <zeta^2> = 2/9, <kappa^2> = 4/81;
- the Schwinger-Dyson sums against fields recomputed by the pinned field.
"""
import numpy as np
import pytest


def _rand_state(L, rng):
    s = rng.standard_normal((L ** 3, 3))
    return s / np.linalg.norm(s, axis=1)[:, None]


def _zeta_det(L, s):
    """zeta[x, mu] as det[s_{x+e_mu}, s_x, s_{x-e_mu}] on the (z, y, x) grid."""
    g = s.reshape(L, L, L, 3)
    out = np.zeros((L, L, L, 3))
    for mu, ax in enumerate((2, 1, 0)):  # mu = x, y, z axes of the grid
        sp = np.roll(g, -1, axis=ax)
        sm = np.roll(g, +1, axis=ax)
        out[..., mu] = np.linalg.det(np.stack([sp, g, sm], axis=-2))
    return out


@pytest.mark.parametrize("L", [4, 6])
def test_fourier_sums_match_fft(orc, L):
    rng = np.random.default_rng(100 + L)
    sa, sb = _rand_state(L, rng), _rand_state(L, rng)
    rec = orc.overlaps(L, sa, sb)
    N = L ** 3
    ga, gb = sa.reshape(L, L, L, 3), sb.reshape(L, L, L, 3)
    for al in range(3):
        for be in range(3):
            q = ga[..., al] * gb[..., be]
            F = np.conj(np.fft.fftn(q)) / N  # exp(+i k.x) convention
            n = al * 3 + be
            assert abs(rec["q0"][n] - F[0, 0, 0].real) < 1e-14
            for d, idx in enumerate([(0, 0, 1), (0, 1, 0), (1, 0, 0)]):
                assert abs(rec["qk_re"][d, n] - F[idx].real) < 1e-14
                assert abs(rec["qk_im"][d, n] - F[idx].imag) < 1e-14
    kappa = _zeta_det(L, sa) * _zeta_det(L, sb)
    for mu in range(3):
        F = np.conj(np.fft.fftn(kappa[..., mu])) / N
        assert abs(rec["cg0"][mu] - F[0, 0, 0].real) < 1e-14
        for d, idx in enumerate([(0, 0, 1), (0, 1, 0), (1, 0, 0)]):
            assert abs(rec["cgk_re"][d, mu] - F[idx].real) < 1e-14
            assert abs(rec["cgk_im"][d, mu] - F[idx].imag) < 1e-14


def test_chirality_worked_example(orc):
    """Three spins along x: s_{x-e} = e1, s_x = e2, s_{x+e} = e3 gives
    zeta = e3 . (e2 x e1) = -1; the same with replica b gives kappa = +1."""
    L, N = 4, 64
    s = np.tile([0.0, 0.0, 1.0], (N, 1))
    i = 5  # (x=1, y=1, z=0)
    s[i - 1] = [1, 0, 0]
    s[i] = [0, 1, 0]
    s[i + 1] = [0, 0, 1]
    z = _zeta_det(L, s)
    assert z[0, 1, 1, 0] == pytest.approx(-1.0)
    rec = orc.overlaps(L, s, s)
    kappa = z ** 2
    np.testing.assert_allclose(rec["cg0"], kappa.reshape(-1, 3).mean(axis=0), atol=1e-15)
    assert rec["cg0"][0] >= 1.0 / N


def test_infinite_temperature_closed_forms(orc):
    L = 6
    rng = np.random.default_rng(7)
    qq, q2, z2, k2 = [], [], [], []
    for _ in range(40):
        sa, sb = _rand_state(L, rng), _rand_state(L, rng)
        qx = (sa * sb).sum(axis=1)
        qq.append((qx ** 2).mean())
        q2.append(((sa[:, :, None] * sb[:, None, :]) ** 2).sum(axis=(1, 2)).mean())
        za, zb = _zeta_det(L, sa), _zeta_det(L, sb)
        z2.append((za ** 2).mean())
        k2.append(((za * zb) ** 2).mean())
        rec = orc.overlaps(L, sa, sb)
        # q(0) = trace of the overlap tensor
        assert abs(np.trace(rec["q0"].reshape(3, 3)) - qx.mean()) < 1e-15
    for vals, exact in ((qq, 1 / 3), (q2, 1.0), (z2, 2 / 9), (k2, 4 / 81)):
        vals = np.array(vals)
        assert abs(vals.mean() - exact) < 5 * vals.std() / np.sqrt(len(vals)) + 1e-12


def test_sd_sums(orc):
    L = 4
    rng = np.random.default_rng(8)
    M = rng.standard_normal((3, L ** 3, 3, 3))
    s = _rand_state(L, rng)
    h = orc.local_fields(L, M, s)
    sh = (s * h).sum(axis=1)
    sd1, sd2 = orc.sd_sums(L, M, s)
    assert abs(sd1 - sh.sum()) < 1e-12
    assert abs(sd2 - ((h * h).sum(axis=1) - sh ** 2).sum()) < 1e-11
    assert abs(sd1 + 2 * orc.energy(L, M, s)) < 1e-11
