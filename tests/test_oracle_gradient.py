"""Pins of the oracle gradient (reverse mode on the oracle forward) of the
per-step estimate with respect to spinor energies and coefficients:
central finite differences under common random numbers (same walkers, same
tau, same lambda) and three exact invariants:
  * sum_k dE/d eps_k = 0 (a common shift of all eps leaves every
    exp((e_i+e_j-e_a-e_b) tau) unchanged);
  * Euler's relation: the estimate is homogeneous of degree 4 in the occupied
    coefficients and separately in the virtual ones, so
    sum_{occ} Re(conj(C) dE/dC) = 4E and sum_{vir} Re(conj(C) dE/dC) = 4E;
  * phase invariance of each spinor: Im sum_mu conj(C_mu k) dE/dC_mu k = 0.
"""
import numpy as np
import pytest

from oracle.gradient import step_value, step_value_and_grad
from oracle.weights import n_g, tau_lambda
from synth import initial_walkers, make_inputs
from synth.generator import probe_rng


@pytest.fixture(scope="module")
def grad_case():
    inp = make_inputs("C0", n_tau=2)
    wk = initial_walkers(inp)
    Ng = n_g(inp.nuc_xyz, inp.wfn)
    lam = tau_lambda(inp.eps, inp.n_occ)
    taus = np.array([0.3, 1.1])
    parts, val, ge, gc = step_value_and_grad(inp, wk, taus, lam, Ng)
    return inp, wk, Ng, lam, taus, val, ge, gc


def test_eps_gradient_finite_differences(grad_case):
    inp, wk, Ng, lam, taus, val, ge, gc = grad_case
    h = 1e-5
    for k in probe_rng(0).choice(inp.n_sp, size=8, replace=False):
        ep, em = inp.eps.copy(), inp.eps.copy()
        ep[k] += h
        em[k] -= h
        fd = (step_value(inp, wk, taus, lam, Ng, eps=ep) - step_value(inp, wk, taus, lam, Ng, eps=em)) / (2 * h)
        assert abs(fd - ge[k]) <= 1e-6 * np.abs(ge).max()


def test_coeff_gradient_finite_differences(grad_case):
    inp, wk, Ng, lam, taus, val, ge, gc = grad_case
    h = 1e-5
    rng = probe_rng(1)
    for _ in range(8):
        s, mu, k = rng.integers(2), rng.integers(inp.n_b), rng.integers(inp.n_sp)
        for unit, part in ((1.0, "re"), (1j, "im")):
            Cp, Cm = inp.coeffs.copy(), inp.coeffs.copy()
            Cp[s, mu, k] += unit * h
            Cm[s, mu, k] -= unit * h
            fd = (step_value(inp, wk, taus, lam, Ng, coeffs=Cp) - step_value(inp, wk, taus, lam, Ng, coeffs=Cm)) / (2 * h)
            an = gc[s, mu, k].real if part == "re" else gc[s, mu, k].imag
            assert abs(fd - an) <= 1e-6 * np.abs(gc).max()


def test_gradient_invariants(grad_case):
    inp, wk, Ng, lam, taus, val, ge, gc = grad_case
    scale = np.abs(ge).max()
    assert abs(ge.sum()) <= 1e-12 * scale * inp.n_sp
    no = inp.n_occ
    occ = np.sum((inp.coeffs.conj() * gc)[:, :, :no]).real
    vir = np.sum((inp.coeffs.conj() * gc)[:, :, no:]).real
    assert abs(occ - 4 * val) <= 1e-10 * abs(val)
    assert abs(vir - 4 * val) <= 1e-10 * abs(val)
    phase = np.sum(inp.coeffs.conj() * gc, axis=(0, 1)).imag
    assert np.abs(phase).max() <= 1e-10 * np.abs(gc).max()


@pytest.fixture(scope="module")
def breit_grad_case():
    inp = make_inputs("C0", n_tau=2)
    wk = initial_walkers(inp)
    Ng = n_g(inp.nuc_xyz, inp.wfn)
    lam = tau_lambda(inp.eps, inp.n_occ)
    taus = np.array([0.3, 1.1])
    parts, val, ge, gc = step_value_and_grad(inp, wk, taus, lam, Ng, interaction="breit")
    return inp, wk, Ng, lam, taus, val, ge, gc


def test_breit_gradient_finite_differences_and_invariants(breit_grad_case):
    """The same pins for the gradient through the Breit forward (Sec. II, the
    full interaction operator): central differences of the oracle's Breit
    step along eps and coefficient probes, the eps-shift invariance, Euler's
    degree-4 relations and the phase invariance (the alpha matrices act on
    the components, not on the orbitals, so all of them still hold), and the
    gradient differs from the Coulomb one."""
    inp, wk, Ng, lam, taus, val, ge, gc = breit_grad_case
    h = 1e-5
    rng = probe_rng(2)
    for k in rng.choice(inp.n_sp, size=6, replace=False):
        ep, em = inp.eps.copy(), inp.eps.copy()
        ep[k] += h
        em[k] -= h
        fd = (step_value(inp, wk, taus, lam, Ng, eps=ep, interaction="breit")
              - step_value(inp, wk, taus, lam, Ng, eps=em, interaction="breit")) / (2 * h)
        assert abs(fd - ge[k]) <= 1e-6 * np.abs(ge).max()
    for _ in range(6):
        s, mu, k = rng.integers(2), rng.integers(inp.n_b), rng.integers(inp.n_sp)
        for unit, part in ((1.0, "re"), (1j, "im")):
            Cp, Cm = inp.coeffs.copy(), inp.coeffs.copy()
            Cp[s, mu, k] += unit * h
            Cm[s, mu, k] -= unit * h
            fd = (step_value(inp, wk, taus, lam, Ng, coeffs=Cp, interaction="breit")
                  - step_value(inp, wk, taus, lam, Ng, coeffs=Cm, interaction="breit")) / (2 * h)
            an = gc[s, mu, k].real if part == "re" else gc[s, mu, k].imag
            assert abs(fd - an) <= 1e-6 * np.abs(gc).max()
    assert abs(ge.sum()) <= 1e-12 * np.abs(ge).max() * inp.n_sp
    no = inp.n_occ
    occ = np.sum((inp.coeffs.conj() * gc)[:, :, :no]).real
    vir = np.sum((inp.coeffs.conj() * gc)[:, :, no:]).real
    assert abs(occ - 4 * val) <= 1e-10 * abs(val)
    assert abs(vir - 4 * val) <= 1e-10 * abs(val)
    assert np.abs(np.sum(inp.coeffs.conj() * gc, axis=(0, 1)).imag).max() <= 1e-10 * np.abs(gc).max()
    _, _, ge_c, gc_c = step_value_and_grad(inp, wk, taus, lam, Ng)
    assert np.abs(gc - gc_c).max() > 1e-4 * np.abs(gc).max()
