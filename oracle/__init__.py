"""FP64 CPU oracle for the DF-DSRG-PT2 virtual natural-orbital pass.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
runs this code; only the tests, the smoke check and the benchmark's CPU
baseline do.  It shares no code with the HIP path.

Modules:
  dsrg_pt2   amplitudes (Eq. A7), PT2 energy, virtual 1-RDM (Eq. A9),
             natural orbitals (Eq. 8), truncation (Eqs. 9-10 and the
             near-degeneracy rule of Sec. 2), recanonicalization and the
             additive correction (Eq. 11)
  screening  (added with the learned pair screen)
"""
from . import dsrg_pt2  # noqa: F401
