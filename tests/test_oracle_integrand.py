"""Pins of the oracle's integrand (Sec. III) against Eq. FinalMP2 and the
mathematics of the Green's functions.

Grid model: space is replaced by K points, the two 1/r factors by a
symmetric positive matrix V and the spinor values by arbitrary complex
numbers.  Then the integrand summed over all K^4 point quadruples at a fixed
tau must equal, exactly,
    -(1/2) sum_{ijab} (ia|jb)_V [(ai|bj)_V - (bi|aj)_V] exp((e_i+e_j-e_a-e_b) tau)
with (pq|rs)_V = sum_xy rho_pq(x) V_xy rho_rs(y), rho_pq = phi_p^dagger phi_q --
the Laplace-transformed Eq. FinalMP2 written as brute-force orbital sums.
"""
import itertools

import numpy as np
import pytest
import torch

from oracle import integrand as itg
from oracle.weights import n_g, pair_weight, tau_lambda
from synth import initial_walkers, make_inputs


def _grid(rng, K, no, nv, nr=False):
    n = no + nv
    if nr:
        psi = rng.standard_normal((K, n // 2))
        phi = np.zeros((K, 4, n), dtype=complex)
        phi[:, 0, 0::2] = psi
        phi[:, 1, 1::2] = psi
    else:
        phi = rng.standard_normal((K, 4, n)) + 1j * rng.standard_normal((K, 4, n))
    e_occ = np.sort(rng.uniform(-3.0, -0.5, no // 2)).repeat(2)
    e_vir = np.sort(rng.uniform(0.2, 5.0, nv // 2)).repeat(2)
    eps = np.concatenate([e_occ, e_vir])
    A = rng.standard_normal((K, K))
    V = A @ A.T + K * np.eye(K)
    return phi, eps, V


def _grid_sum(phi, eps, V, no, tau, form="trace"):
    K = phi.shape[0]
    ph = torch.from_numpy(phi)
    eo, ev = itg.tau_factors(torch.from_numpy(eps), no, tau)
    Gm = itg.green_matrix(ph[:, :, :no], eo)
    Gp = itg.green_matrix(ph[:, :, no:], ev)
    q = np.array(list(itertools.product(range(K), repeat=4)))
    i1, i2, i3, i4 = (torch.from_numpy(q[:, j]) for j in range(4))
    Vt = torch.from_numpy(V)
    wts = Vt[i1, i2] * Vt[i3, i4]
    if form == "trace":
        D, X = itg.direct_exchange(Gm, Gp, i1, i2, i3, i4)
        return complex((-0.5 * D * wts).sum()), complex((0.5 * X * wts).sum())
    return complex((itg.printed_form(Gm, Gp, i1, i2, i3, i4) * wts).sum())


def _orbital_sums(phi, eps, V, no, tau):
    rho = np.einsum("xcp,xcq->xpq", phi.conj(), phi)
    eri = np.einsum("xpq,xy,yrs->pqrs", rho, V, rho)
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


@pytest.mark.parametrize("tau", [0.0, 0.21, 1.7])
@pytest.mark.parametrize("seed", [0, 1])
def test_grid_model_equals_final_mp2_orbital_sums(tau, seed):
    rng = np.random.default_rng(seed)
    no, nv = 4, 6
    phi, eps, V = _grid(rng, 5, no, nv)
    d, x = _grid_sum(phi, eps, V, no, tau)
    dr, xr = _orbital_sums(phi, eps, V, no, tau)
    scale = abs(dr) + abs(xr)
    assert abs(d - dr) <= 1e-12 * scale
    assert abs(x - xr) <= 1e-12 * scale


def test_grid_model_nonrelativistic_closed_shell():
    """Pure-spin real spinors: the integrand sums to the closed-shell
    textbook form -sum_{ijab spatial} (ia|jb)[2(ia|jb)-(ib|ja)] e^{Delta tau}."""
    rng = np.random.default_rng(7)
    no, nv, tau = 4, 6, 0.4
    phi, eps, V = _grid(rng, 5, no, nv, nr=True)
    d, x = _grid_sum(phi, eps, V, no, tau)
    psi = phi[:, 0, 0::2].real
    e = eps[0::2]
    mo = np.einsum("xp,xq,xy,yr,ys->pqrs", psi, psi, V, psi, psi)
    ref = 0.0
    for i in range(no // 2):
        for j in range(no // 2):
            for a in range(no // 2, e.shape[0]):
                for b in range(no // 2, e.shape[0]):
                    ref -= mo[i, a, j, b] * (2 * mo[i, a, j, b] - mo[i, b, j, a]) * np.exp(
                        (e[i] + e[j] - e[a] - e[b]) * tau)
    assert abs((d + x) - ref) <= 1e-12 * abs(ref)


def test_printed_form_is_not_final_mp2():
    """Negative control: Eq. MCMP2 read literally (vec^T vec, prefactors -2, +1)
    does not reproduce Eq. FinalMP2 for 4x4 spinor blocks; in the
    nonrelativistic limit its direct part is four times too large."""
    rng = np.random.default_rng(11)
    no, nv, tau = 4, 6, 0.3
    phi, eps, V = _grid(rng, 4, no, nv)
    d, x = _grid_sum(phi, eps, V, no, tau)
    lit = _grid_sum(phi, eps, V, no, tau, form="printed")
    assert abs(lit - (d + x)) > 0.1 * abs(d + x)
    phi, eps, V = _grid(rng, 4, no, nv, nr=True)
    d, x = _grid_sum(phi, eps, V, no, tau)
    lit = _grid_sum(phi, eps, V, no, tau, form="printed")
    assert abs(lit - (d + x)) > 0.5 * abs(d + x)


@pytest.fixture(scope="module")
def c0_step():
    inp = make_inputs("C0")
    wk = initial_walkers(inp)
    Ng = n_g(inp.nuc_xyz, inp.wfn)
    lam = tau_lambda(inp.eps, inp.n_occ)
    return inp, wk, Ng, lam


def test_green_functions_hermitian_and_kramers(c0_step):
    inp, wk, Ng, lam = c0_step
    phi = itg.spinor_values(wk.reshape(-1, 3), inp)
    eo, ev = itg.tau_factors(torch.from_numpy(inp.eps), inp.n_occ, 0.8)
    for G in (itg.green_matrix(phi[:, :, :inp.n_occ], eo), itg.green_matrix(phi[:, :, inp.n_occ:], ev)):
        P = G.shape[0]
        M = G.reshape(P * 4, P * 4)
        assert torch.allclose(M, M.conj().T, rtol=0, atol=1e-13 * M.abs().max())
        # Kramers pairs make the 2x2 spin blocks of G(x, x) quaternion-like:
        # G^{La La}(x,x) = G^{Lb Lb}(x,x) for the large component
        assert torch.allclose(G[:, 0, :, 0].diagonal(), G[:, 1, :, 1].diagonal(), atol=1e-12 * M.abs().max())


def test_pair_swap_conjugates_and_electron_swap_invariant(c0_step):
    inp, wk, Ng, lam = c0_step
    taus = [0.37]
    _, pairs = itg.step_estimate(inp, wk, taus, lam, Ng, return_pairs=True)
    base = pairs[0]
    # walkers reversed -> pair (p,q) becomes (m-1-q, m-1-p): p <-> q roles swapped
    m = wk.shape[0]
    _, pr = itg.step_estimate(inp, wk[::-1].copy(), taus, lam, Ng, return_pairs=True)
    P, Q = torch.triu_indices(m, m, 1)
    lookup = {(int(p), int(q)): k for k, (p, q) in enumerate(zip(P, Q))}
    swapped = torch.stack([pr[0][lookup[(m - 1 - int(q), m - 1 - int(p))]] for p, q in zip(P, Q)])
    assert torch.allclose(swapped, base.conj(), rtol=1e-12, atol=1e-14 * base.abs().max())
    # electrons 1 <-> 2 of every pair (and so 3 <-> 4) leave each term unchanged
    _, pe = itg.step_estimate(inp, wk[:, ::-1].copy(), taus, lam, Ng, return_pairs=True)
    assert torch.allclose(pe[0], base, rtol=1e-12, atol=1e-14 * base.abs().max())


def test_inverse_r_cancels_against_weights(c0_step):
    """f / (w_p w_q w_tau) = -(1/2)(D - X) N_g^2 / (g(1) g(2) g(3) g(4) w_tau):
    the 1/r12 and 1/r34 of the integrand cancel those of the pair weights."""
    inp, wk, Ng, lam = c0_step
    tau = 0.6
    res, pairs = itg.step_estimate(inp, wk, [tau], lam, Ng, return_pairs=True)
    phi = itg.spinor_values(wk.reshape(-1, 3), inp)
    eo, ev = itg.tau_factors(torch.from_numpy(inp.eps), inp.n_occ, tau)
    Gm = itg.green_matrix(phi[:, :, :inp.n_occ], eo)
    Gp = itg.green_matrix(phi[:, :, inp.n_occ:], ev)
    m = wk.shape[0]
    P, Q = torch.triu_indices(m, m, 1)
    D, X = itg.direct_exchange(Gm, Gp, 2 * P, 2 * P + 1, 2 * Q, 2 * Q + 1)
    gg = torch.from_numpy(itg.walker_g(wk, inp))
    alt = -0.5 * (D - X) * Ng ** 2 / (gg[P] * gg[Q] * lam * np.exp(-lam * tau))
    assert torch.allclose(alt, pairs[0], rtol=1e-12, atol=0)
    assert abs(float(alt.real.mean()) - float(res[0, 2])) <= 1e-12 * float(alt.abs().mean())


def test_imaginary_part_cancels_over_pairs(c0_step):
    """The imaginary part of a term flips sign with p <-> q, so the sum over
    ordered pairs is real; the unordered average keeps only Re."""
    inp, wk, Ng, lam = c0_step
    _, pairs = itg.step_estimate(inp, wk, [0.5], lam, Ng, return_pairs=True)
    assert pairs[0].imag.abs().max() > 0      # terms are genuinely complex


def test_walker_pair_weight_matches_definition(c0_step):
    inp, wk, Ng, lam = c0_step
    w = pair_weight(wk[:, 0], wk[:, 1], inp.nuc_xyz, inp.wfn, Ng)
    r12 = np.linalg.norm(wk[:, 0] - wk[:, 1], axis=1)
    assert np.allclose(w * Ng * r12, itg.walker_g(wk, inp), rtol=1e-14)
