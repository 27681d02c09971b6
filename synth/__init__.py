"""Seeded synthetic inputs for the MC-MP2 hot path.

This module fabricates what a Dirac--Hartree--Fock run would hand to the
stochastic MP2 step (Sec. II, Eq. (C) of the paper: nuclei, a Cartesian
primitive basis with a kinetic-balance small-component set, Kramers-paired
spinor coefficients and spinor energies) plus the starting walker positions.
It holds none of the MC-MP2 arithmetic: no spinor values, Green's functions,
weights, samplers or energies.  Both the oracle tests and the HIP path read
their inputs from here, and nothing else is shared between them.
"""
from .generator import (  # noqa: F401
    CONFIGS,
    Inputs,
    cartesian_components,
    initial_walkers,
    make_inputs,
)
