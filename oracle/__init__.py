"""CPU oracle — TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct FP64 reference for the staggered-grid
variable-viscosity Stokes velocity smoothers (paper Sec. 2.1, Sec. 3, Sec. 4,
Alg. 2, Sec. 6.4).  Only the tests, the smoke check and the benchmark's CPU
baseline may import it; the HIP library never does, and the two share no
code.  See ``stokes_oracle.c`` for the discrete operator it defines.

Modules:
  * ``oracle.stokes``  — ctypes wrappers over ``liboracle.so`` (operator,
    diagonal, RHS fold, divergence, Jacobi, RBGS, RAS, energy norm, transfers);
  * ``oracle.dense``   — assembled-matrix construction A = B^T W B for tiny
    grids (an independent route to the same operator);
  * ``oracle.mg``      — FP64 V-cycle, coarsest-grid Cholesky solve and the
    refinement loop built from the wrappers.
"""
