"""Pins of the oracle's random-number machinery: Philox4x64-10 against the
library implementation in numpy, the inverse-CDF tau sampler against the
exponential law, and the Laplace identity the tau integration rests on."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import philox
from oracle.sampling import sample_tau


@pytest.mark.parametrize("key", [(0, 0), (5, 7), (2**63 + 11, 2**64 - 1)])
def test_philox_matches_numpy(key):
    k = np.array(key, dtype=np.uint64)
    # numpy's Philox increments its counter before producing a block, so a
    # generator started at counter c - 1 yields block c first.
    for start in (0, 1, 2**40, 2**64 - 3):
        ref = np.random.Philox(key=k, counter=np.array([start, 0, 0, 0], dtype=np.uint64)).random_raw(12)
        ctr = np.zeros((3, 4), dtype=np.uint64)
        for b in range(3):                       # 256-bit counter with carry
            c = start + 1 + b
            ctr[b, 0], ctr[b, 1] = c % 2**64, c // 2**64
        got = philox.philox4x64(ctr, k).reshape(-1)
        assert np.array_equal(got, ref)


def test_philox_high_counter_words_match_numpy():
    k = np.array([3, 9], dtype=np.uint64)
    c = np.array([17, 123456789, 2, 0], dtype=np.uint64)
    bg = np.random.Philox(key=k, counter=c)
    ref = bg.random_raw(4)
    c1 = c.copy()
    c1[0] += np.uint64(1)
    assert np.array_equal(philox.philox4x64(c1, k), ref)


def test_unit_conversion_range():
    u = philox.to_unit(np.array([0, 2**64 - 1, 2**11, 2**63], dtype=np.uint64))
    assert u[0] == 0.0 and u[1] == 1.0 - 2.0 ** -53 and u[2] == 2.0 ** -53 and u[3] == 0.5


def test_tau_sampler_is_exponential():
    lam = 1.7
    taus = np.concatenate([sample_tau((1, 2), s, 8, lam) for s in range(4000)])
    ks = stats.kstest(taus, "expon", args=(0, 1.0 / lam))
    assert ks.pvalue > 1e-3
    assert abs(taus.mean() * lam - 1.0) < 4.0 / math.sqrt(taus.size)


@pytest.mark.parametrize("ratio", [0.5, 1.0, 3.0])
def test_laplace_identity(ratio):
    """int_0^inf exp(-Delta tau) dtau = 1/Delta, estimated as the mean of
    exp(-Delta tau)/w(tau) over inverse-CDF tau (Sec. III), Delta >= lambda/2."""
    lam = 1.3
    delta = ratio * lam
    taus = np.concatenate([sample_tau((9, 1), s, 16, lam) for s in range(3000)])
    q = np.exp(-delta * taus) / (lam * np.exp(-lam * taus))
    mean, se = q.mean(), q.std() / math.sqrt(q.size)
    assert abs(mean - 1.0 / delta) < 3.0 * se + 1e-15
    if ratio == 1.0:
        assert np.allclose(q, 1.0 / lam)   # zero-variance case
