"""Pins of the oracle's parallel-tempering pass (appendix A.1).

- a hand-worked pass where every proposal is accepted, fixing the
  ascending sequential order of the pairs (the order is not stated in the
  paper; the reading taken is ascending, one pass over all pairs);
- the acceptance frequency of a single pair against min(1, exp(Delta))
  (binomial test);
- on a three-temperature toy with fixed energies, the long-run frequency of
  the six slot assignments against the Boltzmann weights prod_k
  exp(-beta_k E_{perm[k]}) that detailed balance implies;
- two temperatures on the two-spin system: each slot's energy law is the
  exact canonical law at its own temperature.
"""
import itertools

import numpy as np
import pytest
from scipy import stats


def test_all_accepted_pass_order(orc):
    beta = np.array([2.0, 1.5, 1.0])
    E = np.array([5.0, 0.0, -5.0])  # chain j's energy; hottest chain coldest slot
    perm = np.array([0, 1, 2], dtype=np.int32)
    acc = orc.pt_pass(beta, E, perm, seed=1, pass_index=0, sample=0, rep=0)
    # pair (0,1): chain 0 (E=5) moves up; pair (1,2): it moves up again
    assert acc == 2
    np.testing.assert_array_equal(perm, [1, 2, 0])


def test_single_pair_acceptance_rate(orc):
    beta = np.array([1.0, 0.5])
    E = np.array([0.0, 1.4])  # Delta = (1 - 0.5) * (0 - 1.4) = -0.7
    n = 20000
    acc = 0
    for p in range(n):
        perm = np.array([0, 1], dtype=np.int32)
        acc += orc.pt_pass(beta, E, perm, seed=9, pass_index=p, sample=3, rep=1)
    assert stats.binomtest(acc, n, np.exp(-0.7)).pvalue > 1e-3


def test_three_level_detailed_balance(orc):
    beta = np.array([1.6, 1.1, 0.7])
    E = np.array([-1.0, 0.3, 1.2])
    perms = list(itertools.permutations(range(3)))
    w = np.array([np.exp(-sum(beta[k] * E[p[k]] for k in range(3))) for p in perms])
    pi = w / w.sum()
    perm = np.array([0, 1, 2], dtype=np.int32)
    counts = dict.fromkeys(perms, 0)
    n = 30000
    for p in range(n):
        orc.pt_pass(beta, E, perm, seed=123, pass_index=p, sample=0, rep=2)
        counts[tuple(int(v) for v in perm)] += 1
    obs = np.array([counts[p] for p in perms], dtype=np.float64)
    # successive passes are correlated; compare with a generous chi-square
    chi2 = ((obs - n * pi) ** 2 / (n * pi)).sum()
    assert chi2 < 60.0, (obs / n, pi)
    np.testing.assert_allclose(obs / n, pi, atol=0.02)


def test_pt_counter_streams_differ(orc):
    """Different passes, samples and replicas draw different uniforms."""
    beta = np.array([1.0, 0.9])
    E = np.array([0.0, 0.7])
    seen = set()
    for args in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        res = []
        for q in range(64):
            perm = np.array([0, 1], dtype=np.int32)
            res.append(orc.pt_pass(beta, E, perm, 5, args[0] * 1000 + q, args[1], args[2]))
        seen.add(tuple(res))
    assert len(seen) == 4


@pytest.mark.slow
def test_two_temperature_two_spin_toy(orc):
    from oracle import OracleEnsemble
    L, N = 4, 64
    M = np.zeros((3, N, 3, 3), dtype=np.float32)
    J = 1.0
    M[0, 0] = J * np.eye(3)
    temps = [0.5, 1.0]
    ens = OracleEnsemble(L, M, temps, 1, seed=2024)
    E_by_slot = [[], []]
    for t in range(6000):
        ens.step(1, 0)
        ens.swap()
        if t >= 50:
            for k in range(2):
                E_by_slot[k].append(ens.E[0, ens.perm[0, k]])
    for k, T in enumerate(temps):
        b = 1.0 / T
        Es = np.array(E_by_slot[k])
        cdf = lambda x: (np.exp(b * J) - np.exp(-b * np.clip(x, -J, J))) / (2 * np.sinh(b * J))
        assert stats.kstest(Es[::3], cdf).pvalue > 1e-3
