"""One disorder sample simulated by the FP64 oracle, with the semantics of the
GPU library's step / swap / measure calls.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A sample has T temperatures (ascending) and R replicas, i.e. R*T chains.
Chain (r, j) starts at temperature slot j.  perm[r][k] is the chain index j
now at slot k; parallel tempering permutes these labels and never moves
spins (appendix A.1).  One Monte Carlo step of the paper (Sec. III) is
step(1, L) followed by swap().
"""
import numpy as np

from . import oracle as O


class OracleEnsemble:
    def __init__(self, L, couplings, temps, n_replicas, seed, sample=0, spins=None, row_or=False):
        self.L = int(L)
        self.N = self.L ** 3
        self.M = np.ascontiguousarray(np.asarray(couplings, dtype=np.float32)
                                      .astype(np.float64).reshape(3, self.N, 3, 3))
        self.temps = np.asarray(temps, dtype=np.float64)
        self.beta = 1.0 / self.temps
        self.T = len(self.temps)
        self.R = int(n_replicas)
        self.seed = int(seed)
        self.row_or = bool(row_or)   # overrelaxation in the row order (oracle.row_sweep)
        self.sample = int(sample)
        self.hb_sweeps = 0
        self.pt_passes = 0
        self.perm = np.tile(np.arange(self.T, dtype=np.int32), (self.R, 1))
        if spins is None:
            self.spins = np.stack([np.stack([O.init_spins(self.L, self.seed, self.sample, j, r)
                                             for j in range(self.T)]) for r in range(self.R)])
        else:
            self.spins = np.ascontiguousarray(np.asarray(spins, dtype=np.float64)
                                              .reshape(self.R, self.T, self.N, 3))
        self.E = np.zeros((self.R, self.T))
        self.update_energies()

    def slot_of(self, r, j):
        return int(np.nonzero(self.perm[r] == j)[0][0])

    def update_energies(self):
        for r in range(self.R):
            for j in range(self.T):
                self.E[r, j] = O.energy(self.L, self.M, self.spins[r, j])

    def _chain_sweeps(self, r, j, n_hb, n_or):
        k = self.slot_of(r, j)
        s = self.spins[r, j]
        for n in range(n_hb):
            O.sweep(self.L, self.M, s, 1, self.beta[k], self.seed,
                    self.hb_sweeps + n, self.sample, k, r)
        for _ in range(n_or):
            if self.row_or:
                O.row_sweep(self.L, self.M, s)
            else:
                O.sweep(self.L, self.M, s, 0, self.beta[k], self.seed, 0,
                        self.sample, k, r)

    def step(self, n_hb, n_or, pool=None):
        """n_hb heat-bath sweeps then n_or overrelaxation sweeps, every chain.
        Chains are independent within a step; with a thread pool (the C
        calls release the GIL) they run concurrently, same result."""
        jobs = [(r, j) for r in range(self.R) for j in range(self.T)]
        if pool is None:
            for r, j in jobs:
                self._chain_sweeps(r, j, n_hb, n_or)
        else:
            list(pool.map(lambda rj: self._chain_sweeps(rj[0], rj[1], n_hb, n_or), jobs))
        self.hb_sweeps += n_hb
        self.update_energies()

    def swap(self):
        acc = 0
        for r in range(self.R):
            acc += O.pt_pass(self.beta, self.E[r], self.perm[r], self.seed,
                             self.pt_passes, self.sample, r)
        self.pt_passes += 1
        return acc

    def measure(self):
        """Records ordered by (slot k, pair a < b), as dicts."""
        out = []
        sd = {}
        for r in range(self.R):
            for j in range(self.T):
                sd[(r, j)] = O.sd_sums(self.L, self.M, self.spins[r, j])
        for k in range(self.T):
            for a in range(self.R):
                for b in range(a + 1, self.R):
                    ja, jb = int(self.perm[a, k]), int(self.perm[b, k])
                    rec = O.overlaps(self.L, self.spins[a, ja], self.spins[b, jb])
                    rec.update(sample=self.sample, tslot=k, rep_a=a, rep_b=b,
                               beta=self.beta[k], E_a=self.E[a, ja], E_b=self.E[b, jb],
                               sd1_a=sd[(a, ja)][0], sd2_a=sd[(a, ja)][1],
                               sd1_b=sd[(b, jb)][0], sd2_b=sd[(b, jb)][1])
                    out.append(rec)
        return out

    def spins_at_slot(self, r, k):
        return self.spins[r, int(self.perm[r, k])]
