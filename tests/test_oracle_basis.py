"""Pins of the oracle's basis-function values (Sec. II: the basis expansion
of Eq. (C) over Cartesian primitive Gaussians, and kinetic balance, which
builds the small-component set from derivatives of the large-component one).

Each test compares ``oracle.basis.basis_values`` with something it does not
compute itself:

* unit L2 norm of every Cartesian component up to l = 4 with the closed-form
  normalisation (2a/pi)^(3/4) (4a)^(l/2) / sqrt((2lx-1)!! (2ly-1)!! (2lz-1)!!),
  integrated by Gauss-Hermite quadrature (exact for polynomial x Gaussian);
* two-centre overlaps of s ... f primitives on distinct centres against the
  Obara-Saika recursion of the input generator, integrated on a product
  Gauss-Hermite grid around each product Gaussian's centre;
* the kinetic-balance span: every derivative d/dx_d of a large-component
  primitive (written out by the product rule here) is reproduced exactly by
  a least-squares combination of the small-component values at random points.

A wrong Cartesian power, a swapped axis or a flipped (x - A) sign in
``basis_values`` changes one of these integrals or leaves a residual.
"""
import math

import numpy as np
import pytest

from oracle.basis import basis_values
from synth import cartesian_components, make_inputs
from synth.generator import overlap_matrix, primitive_norm


def _odd_double_factorial(n):
    out = 1
    for k in range(1, 2 * n, 2):
        out *= k
    return out


def _closed_form_norm(a, lxyz):
    lx, ly, lz = lxyz
    L = lx + ly + lz
    df = _odd_double_factorial(lx) * _odd_double_factorial(ly) * _odd_double_factorial(lz)
    return (2 * a / math.pi) ** 0.75 * (4 * a) ** (L / 2) / math.sqrt(df)


def _grid(centre, p, n):
    """Product Gauss-Hermite nodes and weights for int f(r) exp(-p |r - centre|^2) d^3r."""
    t, w = np.polynomial.hermite.hermgauss(n)
    x = t / math.sqrt(p)
    wx = w / math.sqrt(p)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    W = (wx[:, None, None] * wx[None, :, None] * wx[None, None, :]).ravel()
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) + centre
    return pts, W


def test_unit_norm_of_every_cartesian_component_up_to_l4():
    centre = np.array([0.3, -1.1, 0.7])
    for a in (0.07, 1.3, 250.0):
        for l in range(5):
            comps = np.array(cartesian_components(l), dtype=np.int32)
            n = comps.shape[0]
            norms = np.array([_closed_form_norm(a, c) for c in comps])
            pts, W = _grid(centre, 2 * a, 12)
            chi = basis_values(pts, np.tile(centre, (n, 1)), np.full(n, a), comps, norms)
            # chi^2 = N^2 poly exp(-2 a r^2): divide the Gaussian out, the nodes carry it
            g = np.exp(-2 * a * np.sum((pts - centre) ** 2, axis=1))
            integral = (W[:, None] * chi ** 2 / g[:, None]).sum(axis=0)
            assert np.max(np.abs(integral - 1.0)) < 1e-12, (a, l, integral)


def _check_overlaps(xyz, alpha, lxyz, norm, picks):
    S = overlap_matrix(xyz, alpha, lxyz, norm)
    worst, big = 0.0, 0
    for i, j in picks:
        a, b = alpha[i], alpha[j]
        p = a + b
        P = (a * xyz[i] + b * xyz[j]) / p
        pts, W = _grid(P, p, 10)
        sel = [i, j]
        chi = basis_values(pts, xyz[sel], alpha[sel], lxyz[sel], norm[sel])
        g = np.exp(-p * np.sum((pts - P) ** 2, axis=1))
        val = float(np.sum(W * chi[:, 0] * chi[:, 1] / g))
        # both primitives have unit norm, so |S_ij| <= 1 sets the scale
        worst = max(worst, abs(val - S[i, j]))
        big += abs(S[i, j]) > 1e-3
    return worst, big


def test_two_centre_overlaps_against_obara_saika():
    """Every Cartesian component of s ... g shells on centres about a bohr
    apart (so that the overlaps are of order one), all pairs."""
    rng = np.random.default_rng(5)
    prims = []
    for l in range(5):
        for _ in range(2):
            A = rng.uniform(-0.8, 0.8, size=3)
            a = float(np.exp(rng.uniform(np.log(0.3), np.log(3.0))))
            for c in cartesian_components(l):
                prims.append((A, a, c))
    xyz = np.array([p[0] for p in prims])
    alpha = np.array([p[1] for p in prims])
    lxyz = np.array([p[2] for p in prims], dtype=np.int32)
    norm = primitive_norm(alpha, lxyz)
    picks = [(i, j) for i in range(len(prims)) for j in range(len(prims))
             if not np.allclose(xyz[i], xyz[j])]
    worst, big = _check_overlaps(xyz, alpha, lxyz, norm, picks)
    assert worst < 1e-12, worst
    assert big > 500


def test_two_centre_overlaps_of_the_workload_basis():
    """Pairs of the 340-spinor workload's primitives (s ... f, exponents 0.05
    ... 5000 on three centres 4.894 bohr apart) on distinct centres."""
    inp = make_inputs("C1")
    rng = np.random.default_rng(6)
    L = inp.prim_lxyz.sum(axis=1)
    diffuse = inp.prim_exp < 2.0
    picks = []
    for la in range(4):
        for lb in range(4):
            ia = np.flatnonzero((L == la) & diffuse)
            ib = np.flatnonzero((L == lb) & diffuse)
            for _ in range(8):
                i, j = int(rng.choice(ia)), int(rng.choice(ib))
                if not np.allclose(inp.prim_xyz[i], inp.prim_xyz[j]):
                    picks.append((i, j))
    worst, big = _check_overlaps(inp.prim_xyz, inp.prim_exp, inp.prim_lxyz, inp.prim_norm, picks)
    assert worst < 1e-12, worst
    assert big > 20


def _derivative(points, centre, a, lxyz, norm, axis):
    """d/dx_axis of N (x-Ax)^lx (y-Ay)^ly (z-Az)^lz exp(-a |r-A|^2) by the product rule."""
    d = points - centre
    e = np.exp(-a * np.sum(d * d, axis=1))
    other = np.ones(points.shape[0])
    for k in range(3):
        if k != axis:
            other = other * d[:, k] ** lxyz[k]
    l = lxyz[axis]
    x = d[:, axis]
    dpoly = (l * x ** (l - 1) if l > 0 else 0.0) - 2 * a * x ** (l + 1)
    return norm * other * dpoly * e


@pytest.mark.parametrize("name", ["C0", "C1"])
def test_kinetic_balance_span(name):
    """(sigma . grad) chi^L lies in the span of the small-component set, so
    each derivative d/dx_d chi^L does; least squares over random points near
    the centre leaves a residual at rounding level."""
    inp = make_inputs(name)
    rng = np.random.default_rng(11)
    nL = inp.n_L
    S_idx = np.arange(nL, inp.n_b)
    worst = 0.0
    for mu in rng.choice(nL, size=min(nL, 40), replace=False):
        A, a = inp.prim_xyz[mu], inp.prim_exp[mu]
        # small-component primitives on the same centre with the same exponent
        same = S_idx[np.all(np.isclose(inp.prim_xyz[S_idx], A), axis=1) & np.isclose(inp.prim_exp[S_idx], a)]
        assert same.size > 0
        pts = A + rng.standard_normal((200, 3)) / math.sqrt(2 * a)
        X = basis_values(pts, inp.prim_xyz[same], inp.prim_exp[same], inp.prim_lxyz[same], inp.prim_norm[same])
        for axis in range(3):
            f = _derivative(pts, A, a, inp.prim_lxyz[mu], inp.prim_norm[mu], axis)
            coef, *_ = np.linalg.lstsq(X, f, rcond=None)
            res = np.linalg.norm(X @ coef - f) / np.linalg.norm(f)
            worst = max(worst, res)
    assert worst < 1e-12, worst


def test_kinetic_balance_span_fails_without_the_l_plus_one_shells():
    """Negative control: with the l+1 shells removed the derivatives of the
    large-component functions leave the span (the test above can fail)."""
    inp = make_inputs("C0")
    rng = np.random.default_rng(3)
    mu = int(np.flatnonzero(inp.prim_lxyz[: inp.n_L].sum(axis=1) == 1)[0])
    A, a, l = inp.prim_xyz[mu], inp.prim_exp[mu], int(inp.prim_lxyz[mu].sum())
    S_idx = np.arange(inp.n_L, inp.n_b)
    same = S_idx[np.all(np.isclose(inp.prim_xyz[S_idx], A), axis=1) & np.isclose(inp.prim_exp[S_idx], a)
                 & (inp.prim_lxyz[S_idx].sum(axis=1) < l + 1)]
    pts = A + rng.standard_normal((200, 3)) / math.sqrt(2 * a)
    X = basis_values(pts, inp.prim_xyz[same], inp.prim_exp[same], inp.prim_lxyz[same], inp.prim_norm[same])
    f = _derivative(pts, A, a, inp.prim_lxyz[mu], inp.prim_norm[mu], 0)
    coef, *_ = np.linalg.lstsq(X, f, rcond=None)
    assert np.linalg.norm(X @ coef - f) / np.linalg.norm(f) > 0.1
