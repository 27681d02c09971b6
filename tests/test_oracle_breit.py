"""Pins of the oracle's Gaunt / Breit integrand (the interaction operator of
Sec. II, which the paper leaves out of its runs and calls straightforward to
add in the MC method).

* The Dirac alpha matrices of Eq. alpha satisfy the Clifford algebra.
* The decomposition g = sum W_{mu nu}(r) s_mu(1) s_nu(2) equals the operator
  of Sec. II built directly on the 16-dimensional two-electron spinor space.
* Grid model: with an arbitrary operator-valued interaction W^{mu nu}_{xy}
  (one 4x4 real matrix per pair of grid points, no symmetry assumed), the
  trace form summed over all point quadruples equals the brute-force orbital
  sums -(1/2) sum_{ijab} (ia|jb) [(ai|bj) - (bi|aj)] e^{Delta tau} with
  (pq|rs) = sum_xy sum_{mu nu} rho^mu_pq(x) W^{mu nu}_xy rho^nu_rs(y),
  rho^mu_pq = phi_p^dagger s_mu phi_q.
* Special cases: Coulomb weights reproduce the Coulomb form; with no small
  component the alpha terms vanish (alpha couples L and S only).
"""
import itertools

import numpy as np
import pytest
import torch

from oracle import integrand as itg
from oracle.weights import n_g, tau_lambda
from synth import initial_walkers, make_inputs


def test_dirac_matrices_clifford_algebra():
    s = itg.dirac_matrices().numpy()
    assert np.allclose(s[0], np.eye(4))
    for k in range(1, 4):
        assert np.allclose(s[k], s[k].conj().T)
        for l in range(1, 4):
            anti = s[k] @ s[l] + s[l] @ s[k]
            assert np.allclose(anti, 2.0 * np.eye(4) * (k == l))
    # alpha_1 alpha_2 alpha_3 = i (Sigma_z-like) block-diagonal: product of the
    # three is i times the 4x4 identity in the Dirac representation's blocks
    prod = s[1] @ s[2] @ s[3]
    assert np.allclose(prod, 1j * np.block([[np.zeros((2, 2)), np.eye(2)], [np.eye(2), np.zeros((2, 2))]]))


@pytest.mark.parametrize("kind", ["coulomb", "gaunt", "breit"])
def test_weights_reproduce_interaction_operator(kind):
    rng = np.random.default_rng(3)
    r = rng.standard_normal((5, 3))
    W = itg.interaction_weights(torch.from_numpy(r), kind).numpy()
    s = itg.dirac_matrices().numpy()
    for q in range(r.shape[0]):
        rn = np.linalg.norm(r[q])
        g = np.eye(16) / rn
        if kind != "coulomb":
            g = g - sum(np.kron(s[k], s[k]) for k in range(1, 4)) / (2 * rn)
        if kind == "breit":
            ar = sum(r[q, k - 1] * s[k] for k in range(1, 4))
            g = g - np.kron(ar, ar) / (2 * rn ** 3)
        dec = sum(W[q, mu, nu] * np.kron(s[mu], s[nu]) for mu in range(4) for nu in range(4))
        assert np.allclose(dec, g, atol=1e-14, rtol=0)


def _grid(rng, K, no, nv, small=True):
    n = no + nv
    phi = rng.standard_normal((K, 4, n)) + 1j * rng.standard_normal((K, 4, n))
    if not small:
        phi[:, 2:, :] = 0.0
    e_occ = np.sort(rng.uniform(-3.0, -0.5, no // 2)).repeat(2)
    e_vir = np.sort(rng.uniform(0.2, 5.0, nv // 2)).repeat(2)
    W = rng.standard_normal((K, K, 4, 4))  # arbitrary W^{mu nu}_{xy}
    return phi, np.concatenate([e_occ, e_vir]), W


def _trace_sum(phi, eps, W, no, tau):
    K = phi.shape[0]
    ph = torch.from_numpy(phi)
    eo, ev = itg.tau_factors(torch.from_numpy(eps), no, tau)
    Gm = itg.green_matrix(ph[:, :, :no], eo)
    Gp = itg.green_matrix(ph[:, :, no:], ev)
    q = np.array(list(itertools.product(range(K), repeat=4)))
    i1, i2, i3, i4 = (torch.from_numpy(q[:, j]) for j in range(4))
    Wt = torch.from_numpy(W)
    D, X = itg.direct_exchange_general(Gm, Gp, i1, i2, i3, i4, Wt[i1, i2], Wt[i3, i4])
    return complex((-0.5 * D).sum()), complex((0.5 * X).sum())


def _orbital_sums(phi, eps, W, no, tau):
    s = itg.dirac_matrices().numpy()
    rho = np.einsum("xcp,mcd,xdq->xmpq", phi.conj(), s, phi)        # rho^mu_pq(x)
    eri = np.einsum("xmpq,xymn,ynrs->pqrs", rho, W, rho)             # (pq|rs)
    n = eps.shape[0]
    d = x = 0.0
    for i in range(no):
        for j in range(no):
            for a in range(no, n):
                for b in range(no, n):
                    f = np.exp((eps[i] + eps[j] - eps[a] - eps[b]) * tau)
                    d += -0.5 * eri[i, a, j, b] * eri[a, i, b, j] * f
                    x += 0.5 * eri[i, a, j, b] * eri[b, i, a, j] * f
    return d, x


@pytest.mark.parametrize("tau", [0.0, 0.37, 1.9])
@pytest.mark.parametrize("seed", [0, 1])
def test_grid_model_operator_interaction_equals_orbital_sums(tau, seed):
    rng = np.random.default_rng(100 + seed)
    no, nv = 4, 6
    phi, eps, W = _grid(rng, 4, no, nv)
    d, x = _trace_sum(phi, eps, W, no, tau)
    dr, xr = _orbital_sums(phi, eps, W, no, tau)
    scale = abs(dr) + abs(xr)
    assert abs(d - dr) <= 1e-12 * scale
    assert abs(x - xr) <= 1e-12 * scale


def test_coulomb_weights_reproduce_coulomb_form():
    inp = make_inputs("C0")
    wk = initial_walkers(inp)
    lam, Ng = tau_lambda(inp.eps, inp.n_occ), n_g(inp.nuc_xyz, inp.wfn)
    m = wk.shape[0]
    phi = itg.spinor_values(wk.reshape(2 * m, 3), inp)
    eo, ev = itg.tau_factors(torch.as_tensor(inp.eps), inp.n_occ, 0.6)
    Gm = itg.green_matrix(phi[:, :, :inp.n_occ], eo)
    Gp = itg.green_matrix(phi[:, :, inp.n_occ:], ev)
    P, Q = torch.triu_indices(m, m, offset=1)
    i1, i2, i3, i4 = 2 * P, 2 * P + 1, 2 * Q, 2 * Q + 1
    r12v = torch.from_numpy(wk[:, 0] - wk[:, 1])
    W = itg.interaction_weights(r12v, "coulomb")
    D, X = itg.direct_exchange_general(Gm, Gp, i1, i2, i3, i4, W[P], W[Q])
    D0, X0 = itg.direct_exchange(Gm, Gp, i1, i2, i3, i4)
    r = torch.linalg.norm(r12v, dim=-1)
    c = 1.0 / (r[P] * r[Q])
    assert torch.allclose(D, D0 * c, rtol=1e-13, atol=0)
    assert torch.allclose(X, X0 * c, rtol=1e-13, atol=0)
    # and the estimator's Gaunt / Breit parts differ from the Coulomb one
    e0 = itg.step_estimate(inp, wk, [0.6], lam, Ng)
    for kind in ("gaunt", "breit"):
        e1 = itg.step_estimate(inp, wk, [0.6], lam, Ng, interaction=kind)
        assert torch.max(torch.abs(e1 - e0)) > 1e-6 * torch.max(torch.abs(e0))


@pytest.mark.parametrize("kind", ["gaunt", "breit"])
def test_alpha_terms_vanish_without_small_component(kind):
    """alpha_k maps L to S and S to L, so with phi^S = 0 every trace with an
    alpha insertion vanishes and the integrand is the Coulomb one."""
    rng = np.random.default_rng(9)
    K, no, nv, tau = 4, 4, 6, 0.5
    phi, eps, _ = _grid(rng, K, no, nv, small=False)
    pts = rng.standard_normal((K, 3))
    q = np.array([(a, b, c, d) for a, b, c, d in itertools.product(range(K), repeat=4) if a != b and c != d])
    i1, i2, i3, i4 = (torch.from_numpy(q[:, j]) for j in range(4))
    ph = torch.from_numpy(phi)
    eo, ev = itg.tau_factors(torch.from_numpy(eps), no, tau)
    Gm = itg.green_matrix(ph[:, :, :no], eo)
    Gp = itg.green_matrix(ph[:, :, no:], ev)
    r12 = torch.from_numpy(pts[q[:, 0]] - pts[q[:, 1]])
    r34 = torch.from_numpy(pts[q[:, 2]] - pts[q[:, 3]])
    D, X = itg.direct_exchange_general(Gm, Gp, i1, i2, i3, i4, itg.interaction_weights(r12, kind),
                                       itg.interaction_weights(r34, kind))
    Dc, Xc = itg.direct_exchange_general(Gm, Gp, i1, i2, i3, i4, itg.interaction_weights(r12, "coulomb"),
                                         itg.interaction_weights(r34, "coulomb"))
    assert torch.allclose(D, Dc, rtol=1e-13, atol=1e-15 * float(torch.abs(Dc).max()))
    assert torch.allclose(X, Xc, rtol=1e-13, atol=1e-15 * float(torch.abs(Xc).max()))
