"""Host-side statistics of the chain driver: blocking standard error (the
paper's formula, pinned against the oracle's implementation and a direct
computation) and the weighted merge of independent chains."""
import numpy as np

from oracle.blocking import blocking
from paper_2203_05632_amd.chain import ChainResult, blocking_sigma, merge


def test_blocking_sigma_matches_oracle_and_direct_formula():
    rng = np.random.default_rng(4)
    x = np.cumsum(rng.standard_normal(2350)) * 0.01 + rng.standard_normal(2350)   # correlated series
    assert abs(blocking_sigma(x, 100) - blocking(x, 100)[1]) <= 1e-14 * abs(blocking(x, 100)[1])
    means = np.array([x[i * 100:(i + 1) * 100].mean() for i in range(23)])   # incomplete last block dropped
    direct = np.sqrt(np.mean((means - means.mean()) ** 2) / 23)
    assert abs(blocking_sigma(x, 100) - direct) <= 1e-14 * direct
    assert np.isnan(blocking_sigma(x[:150], 100))


def test_merge_weights_chains_by_step_count():
    r1 = ChainResult(1000, np.array([1.0, 2.0, 3.0]), np.array([0.1, 0.2, 0.3]), np.ones(2), np.ones((2, 3, 2)))
    r2 = ChainResult(3000, np.array([2.0, 4.0, 6.0]), np.array([0.05, 0.1, 0.15]), 3 * np.ones(2),
                     3 * np.ones((2, 3, 2)))
    m = merge([r1, r2])
    assert m.steps == 4000
    assert np.allclose(m.mean, 0.25 * r1.mean + 0.75 * r2.mean, rtol=0, atol=1e-15)
    assert np.allclose(m.sigma, np.sqrt((0.25 * r1.sigma) ** 2 + (0.75 * r2.sigma) ** 2), rtol=0, atol=1e-15)
    assert np.allclose(m.grad_eps, 2.5) and np.allclose(m.grad_coeffs, 2.5)
    # equal lengths: plain average, sigma / sqrt(n_chains) for equal errors
    e = merge([ChainResult(500, np.zeros(3), np.full(3, 0.2)), ChainResult(500, np.ones(3), np.full(3, 0.2))])
    assert np.allclose(e.mean, 0.5) and np.allclose(e.sigma, 0.2 / np.sqrt(2))
