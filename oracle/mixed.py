"""The unhybridised 2x2 velocity / Exner-pressure system (test infrastructure).

Follows Sec. 2.2 of the paper (Eq. of the 2x2 system after density
elimination): the velocity lives in the continuous H(div) space W2 with one
dof per interior facet (global orientation +x, +y, +z), and the rigid lid /
ground facets carry no velocity dof (u . n = 0 there).  The matrix is
assembled from the cell matrices of ``local`` by the sign map between
outward-flux broken dofs and globally oriented dofs.  The velocity-pressure
block includes the facet term <[[theta* w]] {{Pi}}> of the form g, which
vanishes when theta* is single valued on every facet.  On the cubed sphere the
global orientation of a vertical facet is that of its edge (the normal leaves
the first column of the edge); the velocity block then carries the Coriolis
term, which the lumped mass leaves out.

The right-hand side of the continuous problem is obtained from the broken one
by R_u(F) = sum over the two cells K of F of s_{K,F} r^b_{K,F}, the
transformation between the two bases (Sec. 2.4).

Parity: the exact solve by sparse LU is the definition of the answer; it is
pinned by a dense solve on tiny meshes, by the equivalence with the
hybridised solution and by discrete conservation (tests).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import BoxMesh


class MixedSystem:
    def __init__(self, mesh: BoxMesh, loc: dict, prob):
        self.mesh = mesh
        nf = mesh.ntrace
        interior = ~mesh.boundary
        self.udof = -np.ones(nf, np.int64)
        self.udof[interior] = np.arange(int(interior.sum()))
        self.nu = int(interior.sum())
        self.np_ = mesh.ncell
        A = loc["A"]
        cor = loc.get("cor")
        cf, cs = mesh.cell_faces, mesh.cell_sign
        rows_uu, cols_uu, vals_uu, vals_lump = [], [], [], []
        rows_up, cols_up, vals_up = [], [], []
        rows_pu, cols_pu, vals_pu = [], [], []
        cells = np.arange(mesh.ncell)
        for a in range(6):
            ua = self.udof[cf[:, a]]
            ok_a = ua >= 0
            for b in range(6):
                ub = self.udof[cf[:, b]]
                ok = ok_a & (ub >= 0)
                rows_uu.append(ua[ok])
                cols_uu.append(ub[ok])
                vals_uu.append((cs[:, a] * cs[:, b] * A[:, a, b])[ok])
                m = A[:, a, b] if cor is None else A[:, a, b] - cor[:, a, b]
                vals_lump.append((cs[:, a] * cs[:, b] * m)[ok])
            rows_up.append(ua[ok_a])
            cols_up.append(cells[ok_a])
            vals_up.append((cs[:, a] * A[:, a, 6])[ok_a])
            rows_pu.append(cells[ok_a])
            cols_pu.append(ua[ok_a])
            vals_pu.append((cs[:, a] * A[:, 6, a])[ok_a])
        # facet term of g: tau_u dt cp <[[theta* w_F]] {{Pi}}>; on facet F, [[theta* w_F]] =
        # (theta_{K-} - theta_{K+}) / |F| with K- the cell the normal leaves.
        jump = np.zeros(nf)
        coef = prob.tau_u * prob.dt * prob.cp
        for a in range(6):
            np.add.at(jump, cf[:, a], cs[:, a] * loc["thF"][:, a])
        for a in range(6):
            ua = self.udof[cf[:, a]]
            ok = ua >= 0
            rows_up.append(ua[ok])
            cols_up.append(cells[ok])
            vals_up.append(0.5 * coef * jump[cf[:, a]][ok])
        cat = np.concatenate
        self.Muu = sp.csr_matrix((cat(vals_uu), (cat(rows_uu), cat(cols_uu))), shape=(self.nu, self.nu))
        # the velocity block without the Coriolis term, whose row sums give the lumped mass
        self.Muu_nocor = sp.csr_matrix((cat(vals_lump), (cat(rows_uu), cat(cols_uu))), shape=(self.nu, self.nu))
        self.G = sp.csr_matrix((cat(vals_up), (cat(rows_up), cat(cols_up))), shape=(self.nu, self.np_))
        self.Bp = sp.csr_matrix((cat(vals_pu), (cat(rows_pu), cat(cols_pu))), shape=(self.np_, self.nu))
        self.M3pi = sp.diags(A[:, 6, 6])
        self.matrix = sp.bmat([[self.Muu, self.G], [self.Bp, self.M3pi]], format="csc")

    def rhs(self, r_ub_cells: np.ndarray, r_pi_cells: np.ndarray):
        """r_ub_cells: (ncell, 6) broken dual vector; r_pi_cells: (ncell,)."""
        mesh = self.mesh
        Ru = np.zeros(self.nu)
        for a in range(6):
            ua = self.udof[mesh.cell_faces[:, a]]
            ok = ua >= 0
            np.add.at(Ru, ua[ok], (mesh.cell_sign[:, a] * r_ub_cells[:, a])[ok])
        return np.concatenate([Ru, r_pi_cells])

    def solve(self, r_ub_cells, r_pi_cells):
        rhs = self.rhs(r_ub_cells, r_pi_cells)
        sol = spla.splu(self.matrix).solve(rhs)
        return sol[: self.nu], sol[self.nu :]

    def residual(self, u, pi, r_ub_cells, r_pi_cells):
        rhs = self.rhs(r_ub_cells, r_pi_cells)
        return np.linalg.norm(rhs - self.matrix @ np.concatenate([u, pi])) / np.linalg.norm(rhs)

    def backward_error(self, u, pi, r_ub_cells, r_pi_cells):
        """Componentwise backward error max_i |r_i| / (|M| |x| + |b|)_i of a candidate solution.

        The rows of the mixed system differ in scale by many orders of magnitude and the
        pressure rows cancel strongly, so the plain relative 2-norm residual of even the exact
        LU solution is far above rounding level; this measure is scale invariant per row.
        """
        rhs = self.rhs(r_ub_cells, r_pi_cells)
        x = np.concatenate([u, pi])
        r = rhs - self.matrix @ x
        return float((np.abs(r) / (abs(self.matrix) @ np.abs(x) + np.abs(rhs))).max())

    def broken_from_continuous(self, u):
        """Outward-flux broken velocity (ncell, 6) of a continuous W2 field (0 on the lid/ground)."""
        mesh = self.mesh
        ub = np.zeros((mesh.ncell, 6))
        for a in range(6):
            ua = self.udof[mesh.cell_faces[:, a]]
            ok = ua >= 0
            ub[ok, a] = mesh.cell_sign[ok, a] * u[ua[ok]]
        return ub
