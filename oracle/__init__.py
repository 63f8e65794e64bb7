"""CPU FP64 oracle for the fast-diagonalization Helmholtz/Laplace solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or calls
this package; only the tests, the smoke check and the benchmark's CPU-baseline leg
do.  It shares no code with the GPU path: it assembles the finite-volume operator
cell by cell from face fluxes and solves the assembled sparse system with plain
library solvers (dense LU, sparse LU, Jacobi-preconditioned CG).

The method of the paper (Section 3, eqs. 23-29) is a direct solver, so its exact
result is simply the solution of the assembled linear system; the oracle is that
definition written out, not a re-implementation of the eigenvalue factorization.

Modules
  fv        grid geometry, 1D operators, 3D cell-by-cell assembly, MAC div/grad
  solvers   dense LU, sparse LU, Jacobi-PCG on the SPD form, Neumann gauge handling
  pressure  the pressure matrix C of eq. 9 (dense at small sizes, and its action)
  stokes    the Stokes system of eq. 8, assembled and bordered, solved by sparse LU

Every function here is pinned by the CPU tests (tests/test_oracle_*.py) against
closed forms, library transforms, brute force and hand-computed fixtures.
"""
