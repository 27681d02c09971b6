"""Samplers of the MC-MP2 estimator (Sec. III).

Test infrastructure: part of the FP64 oracle.

* Imaginary time: inverse-CDF sampling of w(tau) = lambda exp(-lambda tau):
  tau = -ln(1 - u) / lambda with u uniform in [0, 1).
* Electron-pair walkers: Metropolis sampling of w(r1, r2).  The paper names
  only "the Metropolis algorithm"; the proposal adopted here moves both
  electrons of a pair jointly, each coordinate by delta * (2u - 1), and
  accepts iff u_acc < w(new) / w(old).  One proposal per pair per step.

Random numbers come from Philox4x64-10 with key (seed, chain) and counter
(step, pair or tau index, purpose, 0):
    purpose 0 -> uniforms for r1 (x, y, z) and r2 (x) ...
    the six displacement uniforms are words 0..3 of purpose 0 and words 0..1
    of purpose 1; word 2 of purpose 1 is the acceptance uniform;
    purpose 2 word 0 is the uniform behind tau.
"""
from __future__ import annotations

import numpy as np

from . import philox
from .weights import pair_weight


def sample_tau(key, step: int, n_tau: int, lam: float) -> np.ndarray:
    """n_tau imaginary times for MC step `step`."""
    u = philox.draw(key, step, np.arange(n_tau), philox.PURPOSE_TAU)[:, 0]
    return -np.log(1.0 - u) / lam


def metropolis_step(walkers: np.ndarray, w: np.ndarray, key, step: int, delta: float,
                    nuc_xyz, wfn, Ng: float):
    """One Metropolis proposal per electron pair.

    walkers : [m, 2, 3]; w : [m] current pair weights.
    Returns (new_walkers, new_w, accepted[m] bool).
    """
    m = walkers.shape[0]
    pairs = np.arange(m)
    a = philox.draw(key, step, pairs, philox.PURPOSE_MOVE)     # [m, 4]
    b = philox.draw(key, step, pairs, philox.PURPOSE_ACCEPT)   # [m, 4]
    u = np.concatenate([a, b[:, :2]], axis=1).reshape(m, 2, 3)
    shift = delta * (2.0 * u - 1.0)
    trial = walkers + shift
    w_trial = pair_weight(trial[:, 0], trial[:, 1], nuc_xyz, wfn, Ng)
    accept = b[:, 2] < w_trial / w
    new_walkers = np.where(accept[:, None, None], trial, walkers)
    new_w = np.where(accept, w_trial, w)
    return new_walkers, new_w, accept
