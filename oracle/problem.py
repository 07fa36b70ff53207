"""Glue: build every oracle object for one synthetic problem, periodic box or extruded cubed
sphere (test infrastructure)."""

from __future__ import annotations

import numpy as np

from .hybrid import HybridSystem
from .krylov import fgmres
from .local import local_matrices, shell_local_matrices
from .mesh import BoxMesh, TableMesh
from .mixed import MixedSystem
from .precond import COARSE_CHEB, TwoLevel, pressure_operator


def cells_from_soa(r_ub, r_pi):
    """[6][L][ncol] and [L][ncol] -> (ncell, 6) and (ncell,) in cell order k*ncol+col."""
    L, ncol = r_pi.shape
    return np.ascontiguousarray(r_ub.reshape(6, L * ncol).T), r_pi.reshape(L * ncol).copy()


class OracleProblem:
    def __init__(self, prob, *, with_mixed=True, with_precond=True, omega=0.6, n_pre=1,
                 n_post=2, mg_levels=None, omega_p=0.9, mg_pre=1, mg_post=2, mg_coarse_sweeps=6,
                 mg_coarse_cheb=COARSE_CHEB, coarse=True, smoother_patch=False, log=None):
        """log (optional): called with a line after each setup step (for long setups)."""
        say = log or (lambda msg: None)
        self.prob = prob
        if getattr(prob, "geom", "box") == "shell":
            self.mesh = TableMesh(prob.nlev, prob.col_edge, prob.edge_col, prob.edge_lf,
                                  parents=[L.parent for L in prob.levels[1:]])
            self.loc = shell_local_matrices(self.mesh, prob)
        else:
            self.mesh = BoxMesh(prob.nx, prob.ny, prob.nlev, prob.dx, prob.dy, prob.z)
            self.loc = local_matrices(self.mesh, prob)
        say("oracle setup: cell matrices")
        self.hyb = HybridSystem(self.mesh, self.loc)
        say("oracle setup: hybrid system")
        self.mixed = MixedSystem(self.mesh, self.loc, prob) if (with_mixed or with_precond) else None
        say("oracle setup: mixed system")
        self.pc = None
        if with_precond:
            self.H = pressure_operator(self.mixed)
            if mg_levels is None:
                mg_levels = len(prob.levels)
            self.pc = TwoLevel(self.mesh, self.hyb.S, self.H, omega=omega, n_pre=n_pre,
                               n_post=n_post, mg_levels=mg_levels, omega_p=omega_p, mg_pre=mg_pre,
                               mg_post=mg_post, mg_coarse_sweeps=mg_coarse_sweeps,
                               mg_coarse_cheb=mg_coarse_cheb, coarse=coarse,
                               smoother_patch=prob.levels[1].parent if smoother_patch else None)
            say("oracle setup: preconditioner")

    def solve_fgmres(self, B, rtol=1e-8, restart=30, maxit=500, precondition=True):
        M = self.pc if precondition else (lambda r: r)
        return fgmres(lambda x: self.hyb.S @ x, M, B, rtol=rtol, restart=restart, maxit=maxit)
