"""Static condensation onto the trace space (test infrastructure).

Follows Sec. 2.4 of the paper: the hybridised 3x3 block system (Eq. of the
hybridisable system) with its block form [[A, K], [C^T, 0]], the Schur
complement S = C^T A^{-1} K (Eq. of S), the right-hand side
B_lambda = C^T A^{-1} R_X (Eq. of B_lambda) and the local recovery
X = A^{-1}(R_X - K lambda) (Eq. of the recovery).  A^{-1} is applied cell by
cell with ``numpy.linalg.solve``.

Parity: pinned by the dense brute-force solve of the full KKT system on tiny
meshes, by the equivalence of the recovered (u, Pi) with the mixed solution,
by continuity / conservation of the recovered broken velocity and by the
symmetry and definiteness of S in the symmetric special case (tests).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import BoxMesh


class HybridSystem:
    def __init__(self, mesh: BoxMesh, loc: dict):
        self.mesh = mesh
        self.A = loc["A"]
        self.Kc = loc["K"]
        self.Cc = loc["C"]
        n = mesh.ncell
        # Khat_K = [K_K; 0] (7 x 6); A_K^{-1} Khat_K for all cells
        Khat = np.zeros((n, 7, 6))
        Khat[:, :6, :] = self.Kc
        self.AinvK = np.linalg.solve(self.A, Khat)  # (n, 7, 6)
        # S_K = C_K^T [A_K^{-1} Khat_K]_u
        self.S_cell = np.einsum("caf,cag->cfg", self.Cc, self.AinvK[:, :6, :])
        cf = mesh.cell_faces
        rows = np.repeat(cf[:, :, None], 6, axis=2).ravel()
        cols = np.repeat(cf[:, None, :], 6, axis=1).ravel()
        self.S = sp.csr_matrix((self.S_cell.ravel(), (rows, cols)), shape=(mesh.ntrace, mesh.ntrace))
        self.S.sum_duplicates()

    def rhs(self, r_ub_cells, r_pi_cells):
        """B_lambda = C^T A^{-1} R_X."""
        R = np.concatenate([r_ub_cells, r_pi_cells[:, None]], axis=1)
        X = np.linalg.solve(self.A, R[:, :, None])[:, :, 0]
        b = np.einsum("caf,ca->cf", self.Cc, X[:, :6])
        B = np.zeros(self.mesh.ntrace)
        np.add.at(B, self.mesh.cell_faces.ravel(), b.ravel())
        return B

    def recover(self, lam, r_ub_cells, r_pi_cells):
        """X = A^{-1}(R_X - K lambda) -> (u_b (ncell, 6), Pi (ncell,))."""
        lam_c = lam[self.mesh.cell_faces]  # (n, 6)
        R = np.concatenate([r_ub_cells, r_pi_cells[:, None]], axis=1)
        R[:, :6] -= np.einsum("caf,cf->ca", self.Kc, lam_c)
        X = np.linalg.solve(self.A, R[:, :, None])[:, :, 0]
        return X[:, :6], X[:, 6]

    def solve_direct(self, r_ub_cells, r_pi_cells):
        B = self.rhs(r_ub_cells, r_pi_cells)
        lam = spla.splu(self.S.tocsc()).solve(B)
        u_b, pi = self.recover(lam, r_ub_cells, r_pi_cells)
        return lam, u_b, pi, B

    def kkt_dense(self):
        """The full hybridised matrix [[A, K], [C^T, 0]] as a dense array (tiny meshes only)."""
        mesh = self.mesh
        n = mesh.ncell
        nX = 7 * n
        N = nX + mesh.ntrace
        M = np.zeros((N, N))
        for c in range(n):
            M[7 * c : 7 * c + 7, 7 * c : 7 * c + 7] = self.A[c]
            for a in range(6):
                for f in range(6):
                    F = nX + mesh.cell_faces[c, f]
                    M[7 * c + a, F] += self.Kc[c, a, f]
                    M[F, 7 * c + a] += self.Cc[c, a, f]
        return M

    def solve_kkt_dense(self, r_ub_cells, r_pi_cells):
        n = self.mesh.ncell
        rhs = np.zeros(7 * n + self.mesh.ntrace)
        R = np.concatenate([r_ub_cells, r_pi_cells[:, None]], axis=1)
        rhs[: 7 * n] = R.ravel()
        sol = np.linalg.solve(self.kkt_dense(), rhs)
        X = sol[: 7 * n].reshape(n, 7)
        return sol[7 * n :], X[:, :6], X[:, 6]
