"""A whole MC-MP2 run with the oracle (Sec. III): Metropolis walkers,
inverse-CDF tau, the redundant-walker estimator and blocking.

Test infrastructure: part of the FP64 oracle.

Burn-in steps adapt the Metropolis step size toward an acceptance ratio of
one half (multiplying delta by 1.1 or 0.9 after every step) and are excluded
from the averages; delta is frozen afterwards.
"""
from __future__ import annotations

import numpy as np

from .blocking import blocking
from .integrand import step_estimate
from .sampling import metropolis_step, sample_tau
from .weights import n_g, pair_weight, tau_lambda


class Chain:
    def __init__(self, inp, walkers0: np.ndarray, key=(0, 0), delta: float = 0.5):
        self.inp = inp
        self.key = np.asarray(key, dtype=np.uint64)
        self.Ng = n_g(inp.nuc_xyz, inp.wfn)
        self.lam = tau_lambda(inp.eps, inp.n_occ)
        self.walkers = np.array(walkers0, dtype=float)
        self.w = pair_weight(self.walkers[:, 0], self.walkers[:, 1], inp.nuc_xyz, inp.wfn, self.Ng)
        self.delta = float(delta)
        self.step_index = 0
        self.accepted = 0
        self.proposed = 0

    def move(self):
        self.walkers, self.w, acc = metropolis_step(self.walkers, self.w, self.key, self.step_index,
                                                    self.delta, self.inp.nuc_xyz, self.inp.wfn, self.Ng)
        self.accepted += int(acc.sum())
        self.proposed += acc.shape[0]
        return acc

    def burn_in(self, n: int, adapt: bool = True):
        for _ in range(n):
            acc = self.move()
            if adapt:
                self.delta *= 1.1 if acc.mean() > 0.5 else 0.9
            self.step_index += 1

    def run(self, n_steps: int, n_tau: int = None):
        """Returns per-step values [n_steps, 3] (direct, exchange, total)."""
        n_tau = self.inp.n_tau if n_tau is None else n_tau
        out = np.zeros((n_steps, 3))
        for s in range(n_steps):
            self.move()
            taus = sample_tau(self.key, self.step_index, n_tau, self.lam)
            out[s] = step_estimate(self.inp, self.walkers, taus, self.lam, self.Ng).mean(dim=0).numpy()
            self.step_index += 1
        return out


def run_mc(inp, walkers0, n_burn: int = 500, n_steps: int = 2000, key=(0, 0), n_b: int = 100):
    """Full run; returns (I_N, sigma_bar_N, per-step values)."""
    ch = Chain(inp, walkers0, key=key)
    ch.burn_in(n_burn)
    vals = ch.run(n_steps)
    I, s = blocking(vals[:, 2], n_b)
    return I, s, vals
