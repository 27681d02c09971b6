"""FP64 CPU oracle for the stochastic four-component relativistic MP2 step.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP implementation is checked against.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path
(the HIP library and its Python binding) never does.

Every function follows a passage of the paper (Cruz, Garza, Yanai, Hirata,
arXiv 2203.05632) and cites it:

* Eq. FinalMP2 (Sec. II): the second-order energy that the estimator targets;
  computed deterministically by ``mp2`` from McMurchie-Davidson integrals
  (``eri``) for tiny inputs.
* Eq. (C) (Sec. II): spinor values from the basis expansion (``basis``,
  ``integrand``).
* Sec. III, Laplace transform, Eq. MCMP2 and the G+/G- definitions: the
  integrand, in the trace form that Eq. FinalMP2 implies for 4x4 spinor
  Green's functions (``integrand``).
* Sec. III, Eq. basisSet, N_g, Eq. tauWeight and the lambda rule: weight
  functions (``weights``).
* Sec. III, Metropolis and inverse-CDF sampling (``sampling``), with the
  counter-based Philox4x64-10 generator of Salmon et al. (SC'11) (``philox``).
* Eq. redundant: the m-walker pair average (``integrand.step_estimate``).
* Eq. uncertainty: blocking statistics (``blocking``).

Arithmetic is float64 / complex128 throughout.  Library primitives (matrix
products, erf, exp, log) serve as steps; there is no blocking, fusion or
reordering beyond what the definitions state.
"""
