"""Pins of the weight functions, the Metropolis sampler and the blocking
estimate (Sec. III)."""
import math

import numpy as np
import pytest

from oracle import weights
from oracle.blocking import blocking
from oracle.sampling import metropolis_step
from synth import initial_walkers, make_inputs


def test_gaussian_normalisation():
    # (2 z / pi)^(3/4) exp(-z r^2) has unit L2 norm: int N^2 exp(-2 z r^2) = 1
    for z in (0.1, 0.6, 3.0):
        assert abs(weights.s_norm(z) ** 2 * (math.pi / (2 * z)) ** 1.5 - 1.0) < 1e-14


def test_two_centre_coulomb_against_monte_carlo():
    """int int exp(-a|r1-A|^2) exp(-b|r2-B|^2)/r12 by direct sampling of the
    two Gaussians (exact iid draws, no Metropolis)."""
    rng = np.random.default_rng(0)
    for a, b, R in ((0.1, 0.6, 4.894), (0.6, 0.6, 0.0), (0.3, 1.7, 1.5)):
        A = np.zeros(3)
        B = np.array([0.0, 0.0, R])
        n = 2_000_000
        r1 = A + rng.standard_normal((n, 3)) * math.sqrt(1 / (2 * a))
        r2 = B + rng.standard_normal((n, 3)) * math.sqrt(1 / (2 * b))
        q = (math.pi / a) ** 1.5 * (math.pi / b) ** 1.5 / np.linalg.norm(r1 - r2, axis=1)
        mean, se = q.mean(), q.std() / math.sqrt(n)
        ref = weights.coulomb_ss(a, b, R * R)
        assert abs(mean - ref) < 4 * se


def test_ng_against_monte_carlo():
    inp = make_inputs("C1")
    Ng = weights.n_g(inp.nuc_xyz, inp.wfn)
    rng = np.random.default_rng(1)
    # sample r1, r2 from the normalised density g / int g (a mixture of Gaussians)
    comps = []
    for I in range(inp.nuc_xyz.shape[0]):
        c1, z1, c2, z2 = inp.wfn[I]
        comps += [(inp.nuc_xyz[I], z1, c1 * weights.s_norm(z1) * (math.pi / z1) ** 1.5),
                  (inp.nuc_xyz[I], z2, c2 * weights.s_norm(z2) * (math.pi / z2) ** 1.5)]
    mass = np.array([c[2] for c in comps])
    total = mass.sum()
    n = 2_000_000

    def draw():
        k = rng.choice(len(comps), size=n, p=mass / total)
        cen = np.array([comps[j][0] for j in k])
        z = np.array([comps[j][1] for j in k])
        return cen + rng.standard_normal((n, 3)) * np.sqrt(1 / (2 * z))[:, None]

    q = total ** 2 / np.linalg.norm(draw() - draw(), axis=1)
    mean, se = q.mean(), q.std() / math.sqrt(n)
    assert abs(mean - Ng) < 4 * se


def test_metropolis_samples_pair_weight():
    """Stationarity: under w(r1, r2) the mean of h(r1,r2) / (r12 w(r1,r2)) is
    int int h / r12; with h = exp(-a|r1-A|^2) exp(-b|r2-B|^2) that is the
    two-centre Coulomb integral (pinned above by direct sampling)."""
    inp = make_inputs("C0")
    Ng = weights.n_g(inp.nuc_xyz, inp.wfn)
    wk = initial_walkers(inp, m=64)
    w = weights.pair_weight(wk[:, 0], wk[:, 1], inp.nuc_xyz, inp.wfn, Ng)
    a, b = 0.5, 0.9
    A, B = inp.nuc_xyz[0], inp.nuc_xyz[1]
    vals = []
    acc = 0
    for s in range(3500):
        wk, w, ok = metropolis_step(wk, w, (4, 0), s, 0.9, inp.nuc_xyz, inp.wfn, Ng)
        acc += ok.sum()
        if s >= 500:
            h = np.exp(-a * np.sum((wk[:, 0] - A) ** 2, 1)) * np.exp(-b * np.sum((wk[:, 1] - B) ** 2, 1))
            r12 = np.linalg.norm(wk[:, 0] - wk[:, 1], axis=1)
            vals.append(np.mean(h / (r12 * w)))
    I, s = blocking(vals, 100)
    ref = weights.coulomb_ss(a, b, float(np.sum((A - B) ** 2)))
    assert 0.2 < acc / (3500 * 64) < 0.9
    assert abs(I - ref) < 3.5 * s
    assert s < 0.05 * ref


def test_blocking_on_ar1_series():
    """AR(1) x_n = phi x_{n-1} + e_n: the variance of the mean of N values is
    sigma_e^2/(1-phi)^2 / N asymptotically; blocking must recover it, while
    the naive standard error underestimates it."""
    rng = np.random.default_rng(2)
    phi, N = 0.8, 400_000
    e = rng.standard_normal(N)
    x = np.empty(N)
    x[0] = e[0] / math.sqrt(1 - phi ** 2)
    for i in range(1, N):
        x[i] = phi * x[i - 1] + e[i]
    _, sb = blocking(x, 100)
    theory = 1.0 / (1 - phi) / math.sqrt(N)
    assert 0.85 < sb / theory < 1.15
    naive = x.std() / math.sqrt(N)
    assert naive < 0.5 * theory


def test_blocking_formula_small_case():
    v = np.arange(400, dtype=float)
    I, s = blocking(v, 100)
    means = np.array([49.5, 149.5, 249.5, 349.5])
    assert I == 199.5
    assert abs(s - math.sqrt(np.mean((means - 199.5) ** 2)) / 2.0) < 1e-12


def test_lambda_rule():
    inp = make_inputs("C0")
    lam = weights.tau_lambda(inp.eps, inp.n_occ)
    assert lam == 2 * (inp.eps[inp.n_occ] - inp.eps[inp.n_occ - 1])
