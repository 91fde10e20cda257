"""CPU oracle for the SIPDG elliptic solver (TEST INFRASTRUCTURE ONLY).

Plain, slow, FP64 reimplementation of what the GPU library computes, written
from the paper (Karakus, Chalmers, Swirydowicz, Warburton, "GPU acceleration
of a high-order discontinuous Galerkin incompressible flow solver"):

  * ``refelem``  - nodal reference triangle (Warp & Blend nodes, Lagrange basis
                   through an orthonormal Dubiner basis), integrals by
                   collapsed-coordinate Gauss quadrature (Sec. 2.1, Sec. 5.2).
  * ``assemble`` - the SIPDG bilinear form plus lambda times the mass form,
                   assembled by quadrature into a sparse matrix, so that
                   A x is the plain definition of the operator (Eq. INS_SD_5,
                   penalty Eq. Ch2.PenaltyParameter, Eq. ellipticOp1).
  * ``solvers``  - textbook (flexible) preconditioned conjugate gradients with
                   Jacobi, block inverse-mass and p-multigrid preconditioners
                   (Sec. 3).

Only the test-suite, the smoke entry point and the benchmark's CPU-baseline
leg may import this package.  The product library never calls it, and it
never calls the product library: the two share no code.  Inputs come from the
``synth`` generators only.
"""
