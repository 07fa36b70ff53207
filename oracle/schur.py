"""The paper's Configuration 1 (test infrastructure; only the tests, the smoke check and the
benchmark's CPU baseline use it): the unhybridised velocity / Exner-pressure system, solved by a
Krylov method preconditioned by the approximate Schur complement of Sec. 2.3.

The preconditioner replaces the velocity block M2 - Q22 by its lumped (diagonal) form and takes
the three steps of Sec. 2.3 on the resulting block system:
  Step 1  the pressure right-hand side  B = R_Pi - (Q32 + M3rho M3^-1 D) M2lumped^-1 R_u,
  Step 2  an approximate solve of H Pi = B by one pressure multigrid V-cycle (H the approximate
          Schur complement of the same lumped system),
  Step 3  the velocity  u = M2lumped^-1 (R_u - G Pi).
The outer iteration runs on the unapproximated system (Eq. of the 2x2 system), as the paper's
solver does; FGMRES takes the place of its BiCGStab, as everywhere in this project.

The mixed vector is laid out as the library lays it out: the velocity on every facet of the trace
numbering, in the facet's global orientation, the ground and lid facets (no velocity dof) held at
zero, followed by one pressure value per cell.

Parity: with an exact solve of H in Step 2 the three steps are the exact inverse of the lumped
block system (pinned); the Krylov solution converges to the sparse LU solution of the mixed system
(pinned).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .krylov import fgmres
from .precond import lumped_velocity_mass


class MixedOperator:
    """The 2x2 system of Sec. 2.2 on the library's layout (trace-numbered velocity, then cells)."""

    def __init__(self, mixed):
        self.mixed = mixed
        self.interior = np.flatnonzero(~mixed.mesh.boundary)
        self.nt = mixed.mesh.ntrace
        self.nc = mixed.np_
        self.n = self.nt + self.nc

    def compress(self, x):
        return np.concatenate([x[: self.nt][self.interior], x[self.nt :]])

    def expand(self, y):
        out = np.zeros(self.n)
        out[self.interior] = y[: self.mixed.nu]
        out[self.nt :] = y[self.mixed.nu :]
        return out

    def __call__(self, x):
        return self.expand(self.mixed.matrix @ self.compress(x))

    def rhs(self, r_ub_cells, r_pi_cells):
        return self.expand(self.mixed.rhs(r_ub_cells, r_pi_cells))


class ApproximateSchur:
    """Steps 1-3 of Sec. 2.3; ``pressure_solve`` maps B to an approximation of H^-1 B."""

    def __init__(self, mixed, pressure_solve):
        self.op = MixedOperator(mixed)
        self.m2l = lumped_velocity_mass(mixed)
        self.D = sp.csr_matrix(mixed.Bp)  # Q32 + M3rho M3^-1 D, cells x velocity dofs
        self.G = sp.csr_matrix(mixed.G)  # velocity dofs x cells
        self.pressure_solve = pressure_solve

    def __call__(self, r):
        nu = self.op.mixed.nu
        rc = self.op.compress(r)
        r_u, r_pi = rc[:nu], rc[nu:]
        B = r_pi - self.D @ (r_u / self.m2l)  # Step 1
        pi = self.pressure_solve(B)  # Step 2
        u = (r_u - self.G @ pi) / self.m2l  # Step 3
        return self.op.expand(np.concatenate([u, pi]))


def solve_configuration1(mixed, pressure_solve, b, rtol=1e-8, restart=30, maxit=500):
    """FGMRES on the mixed system with the approximate-Schur preconditioner, from zero.
    Returns (x, history, iterations, converged) in the library's layout."""
    pc = ApproximateSchur(mixed, pressure_solve)
    return fgmres(pc.op, pc, b, rtol=rtol, restart=restart, maxit=maxit)
