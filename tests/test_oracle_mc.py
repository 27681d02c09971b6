"""End-to-end pins of the oracle's stochastic estimator: a whole Metropolis /
inverse-CDF run of Eq. redundant must land within 3 standard errors (blocking,
Eq. uncertainty) of the deterministic second-order energy of Eq. FinalMP2
computed from McMurchie-Davidson integrals and an explicit four-index
transformation -- for the direct and exchange parts separately and for the
total.  The nonrelativistic limit is checked against the closed-shell
textbook formula.

The pin workload is the tiny two-nucleus system with basis exponents drawn
from [0.3, 1.2] instead of [0.1, 20]: with random (not self-consistent)
orbitals the wide range puts large orbital amplitude in tight functions that
the Table 1 weight function samples rarely, and the run then needs far more
steps than a unit test can afford (relative uncertainty near 100% after 8000
steps).  With [0.3, 1.2] the uncertainty is about 15-20% of |E2| after 4000
steps of 32 walker pairs.
"""
import numpy as np
import pytest

from oracle import mp2
from oracle.blocking import blocking
from oracle.chain import run_mc
from synth import initial_walkers, make_inputs

pytestmark = pytest.mark.slow


@pytest.mark.parametrize("mode", ["dirac", "nr"])
def test_mc_mean_within_three_sigma_of_final_mp2(mode, torch_threads):
    torch_threads.set_num_threads(1)
    inp = make_inputs("C0", exp_range=(0.3, 1.2), m=32, mode=mode)
    ao = mp2.ao_eri(inp)
    eri = mp2.spinor_eri(inp, ao)
    d_ref, x_ref = mp2.mp2_final_parts(eri, inp.eps, inp.n_occ)
    d_ref, x_ref = d_ref.real, x_ref.real
    e_ref = d_ref + x_ref
    if mode == "nr":
        assert abs(mp2.mp2_closed_shell(inp, ao) - e_ref) < 1e-12 * abs(e_ref)
    _, _, vals = run_mc(inp, initial_walkers(inp), n_burn=300, n_steps=4000)
    for col, ref in ((0, d_ref), (1, x_ref), (2, e_ref)):
        I, s = blocking(vals[:, col], 100)
        assert abs(I - ref) < 3.0 * s, (col, I, s, ref)
        assert s < 0.3 * abs(ref)        # the check has power


def test_mp2_forms_agree_dirac_and_two_component():
    """Eq. FinalMP2 equals the antisymmetrised spin-orbital form for general
    complex spinors, four-component and two-component (zero small part)."""
    for mode in ("dirac", "2c"):
        inp = make_inputs("C0", mode=mode)
        eri = mp2.spinor_eri(inp, mp2.ao_eri(inp))
        e = mp2.mp2_final(eri, inp.eps, inp.n_occ)
        assert abs(e.imag) < 1e-14
        assert abs(e.real - mp2.mp2_spin_orbital(eri, inp.eps, inp.n_occ)) < 1e-12 * abs(e.real)


def test_spinor_eri_hermiticity():
    inp = make_inputs("C0")
    eri = mp2.spinor_eri(inp, mp2.ao_eri(inp))
    # (pq|rs) = (rs|pq) = conj((qp|sr))
    assert np.allclose(eri, eri.transpose(2, 3, 0, 1), atol=1e-13)
    assert np.allclose(eri, eri.transpose(1, 0, 3, 2).conj(), atol=1e-13)


def test_tiny_workload_as_specified(torch_threads):
    """The tiny workload exactly as specified (basis exponents 0.1-20, 16
    walker pairs, one tau per step, 2000 steps after 500 of burn-in): the MC
    mean lies within 3 standard errors of Eq. FinalMP2 for the direct and
    exchange parts and the total.  With random orbitals on this exponent
    range sigma_bar is about 60% of |E2| after 2000 steps, so this check has
    little power; the exponent-narrowed runs above are the powered pins."""
    torch_threads.set_num_threads(1)
    inp = make_inputs("C0")
    assert inp.m == 16 and inp.n_tau == 1
    eri = mp2.spinor_eri(inp, mp2.ao_eri(inp))
    d_ref, x_ref = (v.real for v in mp2.mp2_final_parts(eri, inp.eps, inp.n_occ))
    _, _, vals = run_mc(inp, initial_walkers(inp), n_burn=500, n_steps=2000)
    for col, ref in ((0, d_ref), (1, x_ref), (2, d_ref + x_ref)):
        I, s = blocking(vals[:, col], 100)
        assert abs(I - ref) < 3.0 * s, (col, I, s, ref)
