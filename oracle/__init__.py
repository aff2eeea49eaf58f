"""CPU oracle for the on-lattice higher-order thermal lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 CPU
implementation of what the paper (Shim, "Multidimensional on-lattice
higher-order models in the thermal lattice Boltzmann theory") defines.  Only
the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it.  It shares no code with the HIP library: the two meet only in the
seeded input generators of ``synth_inputs``, which hold none of the method's
arithmetic.

Modules and the passages they follow:

  counting        Formulas (6)-(8), Table 1: partition counting of equations.
  velocity_sets   Symmetry groups and Formulas (9)-(10); Tables 2 and 3; the
                  weight equations, Formulas (3)-(5).
  equilibrium     Maxwellian and dimensionless variables (the paragraph with
                  the update rule), 4th-order Hermite equilibrium (the
                  paragraph around Formula (2) and the one after Formula (8)),
                  moment constraints of Formula (1).
  lbm             The update rule f_i(x+V_i dt, t+dt) = (1-w) f_i + w f_i^eq,
                  initialisation, conservation sums, loss and its gradient.
  riemann         Exact solution of the Riemann problem (shock-tube figure).

Every oracle function is pinned by a test under ``tests/`` against something
other than itself (values printed in the paper, closed forms, brute force,
textbook quadrature, invariants).  Functions without such a pin say
"parity unpinned" in their docstring; at present there are none.
"""
