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


def cell_trace_operator(loc):
    """S_K = C_K^T [A_K^{-1} Khat_K]_u with Khat_K = [K_K; 0] (Eq. of S, one cell) -> (n, 6, 6)."""
    n = loc["A"].shape[0]
    Khat = np.zeros((n, 7, 6))
    Khat[:, :6, :] = loc["K"]
    AinvK = np.linalg.solve(loc["A"], Khat)
    return np.einsum("caf,cag->cfg", loc["C"], AinvK[:, :6, :])


def cell_rhs(loc, r_ub_cells, r_pi_cells):
    """b_K = C_K^T [A_K^{-1} R_K]_u (Eq. of B_lambda, one cell) -> (n, 6) indexed by trace face."""
    R = np.concatenate([r_ub_cells, r_pi_cells[:, None]], axis=1)
    X = np.linalg.solve(loc["A"], R[:, :, None])[:, :, 0]
    return np.einsum("caf,ca->cf", loc["C"], X[:, :6])


def cell_recover(loc, lam_cells, r_ub_cells, r_pi_cells):
    """X_K = A_K^{-1}(R_K - Khat_K lambda_K) (Eq. of the recovery) -> (u_b (n, 6), Pi (n,))."""
    R = np.concatenate([r_ub_cells, r_pi_cells[:, None]], axis=1)
    R[:, :6] -= np.einsum("caf,cf->ca", loc["K"], lam_cells)
    X = np.linalg.solve(loc["A"], R[:, :, None])[:, :, 0]
    return X[:, :6], X[:, 6]


class HybridSystem:
    def __init__(self, mesh: BoxMesh, loc: dict):
        self.mesh = mesh
        self.loc = loc
        self.A = loc["A"]
        self.Kc = loc["K"]
        self.Cc = loc["C"]
        self.S_cell = cell_trace_operator(loc)
        cf = mesh.cell_faces
        rows = np.repeat(cf[:, :, None], 6, axis=2).ravel()
        cols = np.repeat(cf[:, None, :], 6, axis=1).ravel()
        self.S = sp.csr_matrix((self.S_cell.ravel(), (rows, cols)), shape=(mesh.ntrace, mesh.ntrace))
        self.S.sum_duplicates()

    def rhs(self, r_ub_cells, r_pi_cells):
        """B_lambda = C^T A^{-1} R_X."""
        b = cell_rhs(self.loc, r_ub_cells, r_pi_cells)
        B = np.zeros(self.mesh.ntrace)
        np.add.at(B, self.mesh.cell_faces.ravel(), b.ravel())
        return B

    def recover(self, lam, r_ub_cells, r_pi_cells):
        """X = A^{-1}(R_X - K lambda) -> (u_b (ncell, 6), Pi (ncell,))."""
        return cell_recover(self.loc, lam[self.mesh.cell_faces], r_ub_cells, r_pi_cells)

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
