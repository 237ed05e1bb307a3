"""FP64 CPU oracle for the mass-consistent wind solve (TEST INFRASTRUCTURE ONLY).

This package is the slow, plain, obviously-checkable definition of what the
GPU path computes, written from Mandel et al., "Simple finite elements and
multigrid for efficient mass-consistent wind downscaling in a coupled
fire-atmosphere model" (Sec. 2 eqs. (1)-(5); Sec. 3 eqs. (6)-(7)).  It is
used only by the tests, by the package smoke check and by the CPU-baseline
leg of the benchmark.  The product path never imports it, and it imports
nothing from the product path: the two share only the seeded input
generators, which hold none of the method's arithmetic.

Modules
-------
fem        reference hexahedron, 2x2x2 Gauss stiffness, 1-point right-hand
           side, assembly, recovery, divergence check (Sec. 2).
multigrid  coarsening rule, prolongation, Galerkin coarse operators,
           4-colour vertical Gauss-Seidel, V-cycle (Sec. 3).
solve      the discrete solution by direct factorisation or tight CG.
adjoint    gradient of a wind loss through the solve (derived from eqs. (3),
           (5) by the chain rule).

Pinning: every function is checked in tests/test_oracle_*.py against closed
forms, invariants, special cases or brute force (nothing there re-types the
oracle's own formulas).  The actual lambda and u values on real WRF problems
are "parity unpinned": the paper prints no worked example, so they are only
pinned through the invariants and the exactness of the discrete solve.
"""
