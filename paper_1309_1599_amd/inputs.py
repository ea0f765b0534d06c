"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no part of the Monte Carlo method: it only draws the
quenched couplings, temperature grids and test states that both the GPU
library and the CPU oracle take as inputs.

- Couplings: each of the 3N bond matrices has nine iid N(0, 1) entries
  (zero mean, unit variance, as the disorder of Sec. II.A; the matrix is not
  restricted to J*1 + D with D symmetric), drawn from numpy's Philox bit
  generator keyed by (seed, sample) and rounded to FP32.
- Temperatures: evenly spaced or geometric between T_min and T_max
  (Table I uses geometric sequences).
"""
import numpy as np


def rng(seed, *stream):
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([int(seed), *map(int, stream)])))


def gaussian_couplings(L, seed, sample=0):
    """float32 [3][L^3][3][3]; bond (i, i+e_mu) has matrix [mu][i]."""
    g = rng(seed, 3, sample)
    return g.standard_normal((3, L ** 3, 3, 3), dtype=np.float32)


def bimodal_couplings(L, D, seed, sample=0):
    """The paper's family (Sec. II.A): M = J*1 + D_sym, J = +-1 and the six
    independent entries of the symmetric D equal to +-D."""
    g = rng(seed, 4, sample)
    N = L ** 3
    J = g.choice(np.array([-1.0, 1.0], dtype=np.float32), size=(3, N))
    d = g.choice(np.array([-D, D], dtype=np.float32), size=(3, N, 6))
    M = np.zeros((3, N, 3, 3), dtype=np.float32)
    iu = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for n, (a, b) in enumerate(iu):
        M[:, :, a, b] = d[:, :, n]
        M[:, :, b, a] = d[:, :, n]
    M += J[:, :, None, None] * np.eye(3, dtype=np.float32)
    return M


def linear_temps(t_min, t_max, n):
    return np.linspace(t_min, t_max, n)


def geometric_temps(t_min, t_max, n):
    if n == 1:
        return np.array([t_min], dtype=np.float64)
    k = np.arange(n)
    return t_min * (t_max / t_min) ** (k / (n - 1))


def random_spins(N, seed, *stream):
    """Unit vectors uniform on the sphere, float32 [N][3] (renormalised in FP32)."""
    g = rng(seed, 5, *stream)
    v = g.standard_normal((N, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    v = v.astype(np.float32)
    return (v / np.linalg.norm(v, axis=1)[:, None]).astype(np.float32)


# Workload presets (lattice sizes, ensemble shape, step composition).  The
# step is n_hb heat-bath + n_or overrelaxation sweeps + one tempering pass;
# the paper's MCS has n_or = L (Sec. III).  `measure` lists what a
# measurement step records (energies always): the L = 8 workload takes
# E, q(0) and q(k_min) every step, the L = 64 one the q(k_min) Fourier sums
# and the chirality every 10 steps.
C5_TEMPS = {8: 16, 12: 18, 16: 20, 24: 24, 32: 28, 48: 32}

PRESETS = {
    "L8": dict(L=[8], temps=("linear", 0.5, 2.0, 8), R=2, n_hb=1, n_or=8, measure_every=1,
               measure=("overlap",), seed=130915991),
    "L16": dict(L=[16], temps=("geometric", 0.5, 2.0, 16), R=2, n_hb=1, n_or=16,
                measure_every=0, seed=130915992),
    "L32x64": dict(L=[32] * 64, temps=("geometric", 0.6, 1.8, 24), R=4, n_hb=1, n_or=32,
                   measure_every=0, seed=130915993),
    "L64x8": dict(L=[64] * 8, temps=("geometric", 0.6, 1.6, 32), R=4, n_hb=1, n_or=64,
                  measure_every=10, measure=("overlap", "chiral"), seed=130915994),
    "mixedL": dict(L=[L for L in (8, 12, 16, 24, 32, 48) for _ in range(16)],
                   temps=("geometric", 0.6, 1.8, None), R=2, n_hb=1, n_or=None,
                   measure_every=0, seed=130915995),
}


def preset_temps(p, L):
    kind, lo, hi, n = p["temps"]
    n = C5_TEMPS[L] if n is None else n
    return linear_temps(lo, hi, n) if kind == "linear" else geometric_temps(lo, hi, n)


def preset_inputs(name, seed=None):
    """(L list, couplings list, temps list, R, seed) for a preset."""
    p = PRESETS[name]
    seed = p["seed"] if seed is None else seed
    Ls = p["L"]
    cpl = [gaussian_couplings(L, seed, s) for s, L in enumerate(Ls)]
    temps = [preset_temps(p, L) for L in Ls]
    return Ls, cpl, temps, p["R"], seed
