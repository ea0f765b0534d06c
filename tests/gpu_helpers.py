"""Shared helpers of the GPU parity tests: replay one sweep of the oracle on
the state the GPU started from, and the tolerance rule for FP32 spins.

FP32 tolerance.  A spin updated in FP32 from a local field h differs from
the FP64 update by about eps32 * (sum of |terms| of h) / |h|, so the bound
grows where |h| is small.  A site passes if
    |ds| <= 2e-6 * max(1, H_C / |h|),   H_C = 4 (about the median |h| of a
random state with N(0,1) couplings),
and the raw maximum and the count above 2e-6 are reported.  States
equilibrated at the working temperatures have no small fields and meet
2e-6 outright.
"""
import numpy as np

import oracle as O

TOL = 2e-6
H_C = 4.0


def colours(L):
    i = np.arange(L ** 3)
    return (i % L + (i // L) % L + i // (L * L)) % 2


def replay_sweep(L, M, s0, kind, beta, seed, hb_sweep, sample, tslot, rep):
    """One oracle sweep from s0; returns (final spins, |h| at each site's
    update time)."""
    s = np.array(s0, dtype=np.float64, copy=True)
    hmag = np.zeros(L ** 3)
    col = colours(L)
    for c in (0, 1):
        idx = np.nonzero(col == c)[0]
        for i in idx:
            hmag[i] = np.linalg.norm(O.local_field(L, M, s, int(i)))
        O.half_sweep(L, M, s, c, kind, beta, seed, hb_sweep, sample, tslot, rep)
    return s, hmag


def energy_scale(L, M, s):
    """Sum over the 3N bonds of |s_i^T M s_{i+e_mu}|: the magnitude FP32
    rounding of the energy scales with (a random state has |E| far below it)."""
    s = np.asarray(s, np.float64)
    g = s.reshape(L, L, L, 3)
    Mg = np.asarray(M, np.float64).reshape(3, L, L, L, 3, 3)
    tot = 0.0
    for mu, ax in enumerate((2, 1, 0)):
        nb = np.roll(g, -1, axis=ax)
        tot += np.abs(np.einsum("zyxa,zyxab,zyxb->zyx", g, Mg[mu], nb)).sum()
    return tot


def assert_energy_close(E_gpu, L, M, s_ref, rel=1e-6, what=""):
    import oracle as O_
    Eref = O_.energy(L, M, s_ref)
    scale = energy_scale(L, M, s_ref)
    assert abs(E_gpu - Eref) <= rel * scale, f"{what}: E {E_gpu} vs {Eref} (scale {scale:.4g})"


def assert_spins_close(gpu, ref, hmag, what=""):
    d = np.linalg.norm(np.asarray(gpu, np.float64) - ref, axis=1)
    bound = TOL * np.maximum(1.0, H_C / np.maximum(hmag, 1e-30))
    bad = np.nonzero(d > bound)[0]
    msg = (f"{what}: max |ds| = {d.max():.3g}, {np.count_nonzero(d > TOL)} sites above {TOL}, "
           f"{bad.size} beyond the |h|-scaled bound")
    assert bad.size == 0, msg + f"; first at site {bad[0]} (|h| = {hmag[bad[0]]:.3g}, |ds| = {d[bad[0]]:.3g})"
    return d.max(), int(np.count_nonzero(d > TOL))


def assert_resynced_sweep(L, M, before, after, kind, beta, seed, hb_sweep, sample, tslot, rep, sites=None,
                          what=""):
    """One GPU sweep checked site by site on the oracle, re-synced: a
    colour-0 site is updated from the state before the sweep, a colour-1
    site from that state with colour 0 replaced by the GPU's own colour-0
    result (what the GPU's second half-sweep saw), so FP32 differences of
    the first half-sweep do not propagate into the second.  Each site must
    meet |ds| <= TOL * max(1, H_C/|h|).  Returns the largest |ds|."""
    col = colours(L)
    pre = np.asarray(before, np.float64)
    mixed = np.where(col[:, None] == 0, np.asarray(after, np.float64), pre)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    worst = 0.0
    for i in (range(L ** 3) if sites is None else sites):
        state = pre if col[i] == 0 else mixed
        h = O.local_field(L, M, state, int(i))
        if kind == 0:
            ref = O.overrelax_spin(h, state[i])
        else:
            w = O.philox(key, [int(i), hb_sweep, sample, O.ctr3(O.TAG_HB, tslot, rep)])
            ref = O.heatbath_spin(h, beta, O.u23(w[0]), O.u23(w[1]))
        d = float(np.linalg.norm(after[i] - ref))
        hn = float(np.linalg.norm(h))
        assert d <= TOL * max(1.0, H_C / hn), f"{what}: site {int(i)}: |ds| = {d:.3g} at |h| = {hn:.3g}"
        worst = max(worst, d)
    return worst
