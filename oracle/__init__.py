"""CPU FP64 oracle for the hybridised trace solve (test infrastructure only).

This package is the plain, slow reference that the HIP library is checked
against.  It is test infrastructure: only the test suite, the smoke check and
the CPU-baseline leg of the benchmark import it; the product path never does.
It shares no code with the GPU path (only the seeded inputs of ``synth``).

Modules, each following the paper (Betteridge et al., "Hybridised multigrid
preconditioners for a compatible finite element dynamical core"):

* ``mesh``    - the oracle's own dof maps for the periodic extruded box.
* ``local``   - cell matrices of the bilinear forms (Sec. 2.2, Eq. of the eight
  bilinear forms; hybrid forms of Sec. 2.4) by Gauss quadrature of the lowest
  order broken Raviart-Thomas basis.
* ``mixed``   - the unhybridised 2x2 velocity/Exner system (Eq. of the 2x2
  system) assembled in the continuous space and solved by sparse LU.
* ``hybrid``  - static condensation (Eqs. of S, B_lambda and recovery, Sec.
  2.4), the dense KKT brute force and the hybrid solve.
* ``precond`` - lumped approximate Schur operator H (Sec. 2.3), tensor
  product pressure multigrid, LineSmooth (Alg. 1), intergrid operators, the
  scaling Gamma (Eq. of the scaling matrix) and the two-level cycle (Alg. 2).
* ``krylov``  - flexible GMRES (and BiCGStab for the coarse pressure system).
* ``schur``   - the approximate-Schur preconditioner of the unhybridised system (Sec. 2.3).
* ``elimination`` - the elimination of theta' (Sec. 2.1) and rho' (Sec. 2.2) around the 2x2
  solve, their back-substitution and the four-field system they come from.
* ``p1``, ``nn`` - the next-to-lowest order system and the learned coarse correction.

Parity status of every function is listed in its module header.
"""
