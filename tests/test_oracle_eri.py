"""Pins of the oracle's McMurchie-Davidson integrals and Boys function.

* Boys F_n(T) against adaptive quadrature of its defining integral.
* (ss|ss) against the electrostatics of two spherical Gaussian charge clouds,
  Q1 Q2 erf(sqrt(pq/(p+q)) R)/R (a derivation independent of the Hermite scheme).
* Higher angular momenta against centre derivatives of lower ones:
  d/dAx [(x-Ax)^l e^{-a(x-Ax)^2}] = 2a (x-Ax)^{l+1} e^{..} - l (x-Ax)^{l-1} e^{..}.
* Eightfold permutational symmetry.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import eri


@pytest.mark.parametrize("n", [0, 1, 2, 5, 8, 12])
@pytest.mark.parametrize("T", [0.0, 1e-6, 0.3, 4.0, 17.5, 39.9, 40.1, 95.0])
def test_boys_against_quadrature(n, T):
    ref, _ = integrate.quad(lambda t: t ** (2 * n) * math.exp(-T * t * t), 0.0, 1.0, epsabs=0, epsrel=1e-13,
                            limit=200)
    got = eri.boys(n, T)[n]
    assert abs(got - ref) <= 1e-12 * abs(ref) + 1e-300


def _eri_one(prims, quartet):
    xyz = np.array([p[0] for p in prims], dtype=float)
    al = np.array([p[1] for p in prims], dtype=float)
    lx = np.array([p[2] for p in prims], dtype=np.int32)
    nm = np.array([p[3] if len(p) > 3 else 1.0 for p in prims], dtype=float)
    i, j, k, l = quartet
    return eri.eri_pairs(xyz, al, lx, nm, [i, k], [j, l])[0, 1]


def test_ssss_is_gaussian_cloud_electrostatics():
    rng = np.random.default_rng(3)
    for _ in range(20):
        A, B, C, D = rng.normal(size=(4, 3))
        a, b, c, d = np.exp(rng.uniform(-2, 2, size=4))
        prims = [(A, a, (0, 0, 0)), (B, b, (0, 0, 0)), (C, c, (0, 0, 0)), (D, d, (0, 0, 0))]
        got = _eri_one(prims, (0, 1, 2, 3))
        p, q = a + b, c + d
        P, Q = (a * A + b * B) / p, (c * C + d * D) / q
        Q1 = math.exp(-a * b / p * np.sum((A - B) ** 2)) * (math.pi / p) ** 1.5
        Q2 = math.exp(-c * d / q * np.sum((C - D) ** 2)) * (math.pi / q) ** 1.5
        R = float(np.linalg.norm(P - Q))
        w = math.sqrt(p * q / (p + q))
        ref = Q1 * Q2 * (special.erf(w * R) / R if R > 1e-12 else 2.0 * w / math.sqrt(math.pi))
        assert abs(got - ref) <= 1e-12 * abs(ref)


def _raise(prims, idx, axis, h=1e-4):
    """Integral with primitive idx's power along axis raised by one, from the
    centre derivative of the lower one (central differences)."""
    pr = [list(p) for p in prims]

    def val(shift):
        q = [list(p) for p in pr]
        q[idx][0] = np.array(q[idx][0], dtype=float).copy()
        q[idx][0][axis] += shift
        return _eri_one([tuple(x) for x in q], (0, 1, 2, 3))

    dA = (val(h) - val(-h)) / (2 * h)
    l = pr[idx][2][axis]
    lower = 0.0
    if l > 0:
        q = [list(p) for p in pr]
        lq = list(q[idx][2])
        lq[axis] -= 1
        q[idx][2] = tuple(lq)
        lower = _eri_one([tuple(x) for x in q], (0, 1, 2, 3))
    return (dA + l * lower) / (2.0 * pr[idx][1])


@pytest.mark.parametrize("case", [
    # (powers of the four primitives, which primitive to raise, axis)
    (((0, 0, 0), (0, 0, 0), (0, 0, 0), (0, 0, 0)), 0, 0),
    (((1, 0, 0), (0, 0, 0), (0, 0, 0), (0, 0, 0)), 0, 0),
    (((0, 1, 0), (1, 0, 0), (0, 0, 0), (0, 0, 1)), 1, 2),
    (((1, 1, 0), (0, 0, 1), (1, 0, 0), (0, 2, 0)), 3, 1),
    (((2, 0, 0), (0, 1, 1), (0, 0, 2), (1, 0, 1)), 2, 2),
    (((0, 0, 2), (2, 0, 0), (1, 1, 0), (0, 1, 1)), 0, 0),
])
def test_higher_angular_momentum_from_centre_derivatives(case):
    powers, idx, axis = case
    rng = np.random.default_rng(hash(case) % 2**32)
    centres = rng.normal(scale=0.8, size=(4, 3))
    alphas = np.exp(rng.uniform(-1.0, 1.0, size=4))
    prims = [(centres[i], alphas[i], powers[i]) for i in range(4)]
    ref = _raise(prims, idx, axis)
    up = list(powers)
    lp = list(up[idx])
    lp[axis] += 1
    up[idx] = tuple(lp)
    got = _eri_one([(centres[i], alphas[i], up[i]) for i in range(4)], (0, 1, 2, 3))
    assert abs(got - ref) <= 1e-6 * max(1e-3, abs(ref))


def test_eightfold_symmetry():
    rng = np.random.default_rng(5)
    n = 5
    xyz = rng.normal(size=(n, 3))
    al = np.exp(rng.uniform(-1, 1, size=n))
    lx = np.array([(0, 0, 0), (1, 0, 0), (0, 1, 1), (2, 0, 0), (0, 0, 1)], dtype=np.int32)
    full = eri.eri_full(xyz, al, lx, np.ones(n))
    for perm in ("jikl", "ijlk", "klij", "lkji"):
        t = np.einsum("ijkl->" + perm, full)
        assert np.allclose(full, t, rtol=1e-13, atol=1e-15)
    # distributions computed once per unordered pair: also check directly
    pi, pj = [1, 3], [3, 1]
    M = eri.eri_pairs(xyz, al, lx, np.ones(n), pi, pj)
    assert abs(M[0, 0] - M[1, 1]) < 1e-13 * abs(M[0, 0])
