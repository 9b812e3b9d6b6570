"""FP64 CPU oracle for the DF-DSRG-PT2 virtual natural-orbital pass.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
runs this code; only the tests, the smoke check and the benchmark's CPU
baseline do.  It shares no code with the HIP path.

Modules:
  dsrg_pt2   amplitudes (Eq. A7), PT2 energy, virtual 1-RDM (Eq. A9),
             natural orbitals (Eq. 8), truncation (Eqs. 9-10 and the
             near-degeneracy rule of Sec. 2), recanonicalization and the
             additive correction (Eq. 11)
  screening  pair features and rigorous bounds, the FP64 multilayer perceptron,
             its gradient, mean squared error and Adam, used to check the learned
             pair screen (which is not part of the paper's method)
  naf        natural auxiliary functions (compression of the auxiliary basis
             proposed in the paper's conclusions)
  ladder     the density-fitted particle-particle ladder of the high-level step
             (Eq. 6), in the full or the truncated virtual space
  a9_active  the Eq. A9 terms whose amplitudes carry an active particle index
             (zero cumulants, no singles)
  a9_cumulant the first-order singles (Eq. A6) and the remaining Eq. A9 terms:
             the singles and the terms with the two-body density cumulant
"""
from . import a9_active, a9_cumulant, dsrg_pt2, ladder, naf, screening  # noqa: F401
