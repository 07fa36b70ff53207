"""Preconditioner of the trace system (test infrastructure).

Follows the paper:

* Sec. 2.3: the lumped velocity mass matrix, the approximate Schur complement
  H = -(Q32 + M3^rho M3^{-1} D) M2lumped^{-1} G + M3^Pi (Eq. of the elliptic
  pressure system), the block-Jacobi smoother with the column operator H_z
  and relaxation omega (Eq. of the pressure block-Jacobi iteration) inside a
  tensor-product multigrid V-cycle.
* Sec. 2.5: LineSmooth (Alg. 1), prolongation by facet averaging and
  restriction by its transpose (intergrid operators), the row-sum scaling
  Gamma (Eq. of the scaling matrix) and the non-nested two-level cycle
  (Alg. 2).

Readings of the paper taken here (the paper defers the pressure multigrid
details to earlier work and prints one sign that diverges):

* Alg. 1 is applied with the update lambda <- lambda + omega * delta (the
  printed minus sign makes the sweep diverge; the pressure smoother of
  Sec. 2.3 uses the plus sign).
* Lumping: row sums of the assembled continuous velocity block
  (M2 - Q22) in global orientation, over the interior (non-lid) dofs.
* H_z: the diagonal of H plus its couplings to the cells above and below,
  i.e. one tridiagonal block per column.
* Multigrid levels: 2x2 horizontal agglomeration (inside each panel on the
  cubed sphere), no vertical coarsening;
  restriction = sum over the four children, prolongation = injection, coarse
  operators by the Galerkin product R H P; the coarsest level is solved
  approximately with a fixed number of steps: either damped block-Jacobi
  sweeps, or (the default) the Chebyshev semi-iteration preconditioned by
  the same column operator H_z, tuned to eigenvalues of H_z^-1 H in
  [lo, hi] = [0.02, 2].  The upper end holds for every level: H has
  non-positive couplings and positive row sums (H 1 = M3^Pi 1), so
  2 H_z - H, which flips the sign of the horizontal couplings, is
  diagonally dominant and positive definite; the modes below lo are few
  and are left to the Krylov method.
* Prolongation to a facet on the ground or lid is one sided (the value of the
  single adjacent cell), so the restriction weight there is 1 (1/2 elsewhere).

Parity: the smoother, V-cycle and two-level cycle are fixed linear maps;
they are pinned by tests against textbook limits (exact column solves when
the horizontal coupling vanishes, convergence of the stationary iterations,
the divergence of the printed smoother sign), against H 1 = M3^Pi 1 and the
Galerkin identity of the coarse operators, and by brute force on dense
matrices for Gamma.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import BoxMesh


def lumped_velocity_mass(mixed):
    """Row sums of the assembled continuous (M2 - Q22) over interior dofs (without the Coriolis
    term, which has no place in a lumped mass: its rows sum to the rotation of a uniform flow)."""
    return np.asarray(mixed.Muu_nocor.sum(axis=1)).ravel()


def pressure_operator(mixed, m2lumped=None):
    """H = -(Q32 + M3rho M3^-1 D) M2lumped^-1 G + M3Pi (sparse, cells x cells)."""
    if m2lumped is None:
        m2lumped = lumped_velocity_mass(mixed)
    H = -(mixed.Bp @ sp.diags(1.0 / m2lumped) @ mixed.G) + mixed.M3pi
    return sp.csr_matrix(H)


def column_part(H, ncol):
    """Keep the couplings of H between cells of the same column (block tridiagonal here)."""
    Hc = sp.coo_matrix(H)
    keep = (Hc.row % ncol) == (Hc.col % ncol)
    return sp.csr_matrix((Hc.data[keep], (Hc.row[keep], Hc.col[keep])), shape=H.shape)


def agglomeration(nx, ny, nlev):
    """Injection P (fine cells x coarse cells) of the 2x2 horizontal agglomeration."""
    cx, cy = nx // 2, ny // 2
    nf, nc = nx * ny * nlev, cx * cy * nlev
    fine = np.arange(nf)
    k = fine // (nx * ny)
    col = fine % (nx * ny)
    ix, iy = col % nx, col // nx
    coarse = k * cx * cy + (iy // 2) * cx + ix // 2
    return sp.csr_matrix((np.ones(nf), (fine, coarse)), shape=(nf, nc))


def agglomeration_from_parent(parent, ncol_coarse, nlev):
    """Injection P (fine cells x coarse cells) given the coarse column of every fine column."""
    parent = np.asarray(parent, np.int64)
    ncf = parent.shape[0]
    fine = np.arange(ncf * nlev)
    k, col = fine // ncf, fine % ncf
    coarse = k * ncol_coarse + parent[col]
    return sp.csr_matrix((np.ones(fine.shape[0]), (fine, coarse)), shape=(fine.shape[0], ncol_coarse * nlev))


COARSE_CHEB = (0.02, 2.0)  # default interval of the Chebyshev coarsest solve


class PressureMultigrid:
    """coarse_cheb: (lo, hi) for the Chebyshev coarsest solve, or None for damped block-Jacobi
    sweeps; coarse_sweeps: the number of steps either way."""

    def __init__(self, H, nx, ny, nlev, levels=4, omega=0.9, pre=1, post=2, coarse_sweeps=6,
                 coarse_cheb=COARSE_CHEB, parents=None):
        """nx, ny: the periodic box's columns; or ``parents`` (then nx, ny are unused): the coarse
        column of every column, one array per coarsening."""
        self.omega, self.pre, self.post, self.coarse_sweeps = omega, pre, post, coarse_sweeps
        self.coarse_cheb = coarse_cheb
        self.H = [sp.csr_matrix(H)]
        self.P = []
        self.ncol = [H.shape[0] // nlev]
        for lvl in range(1, levels):
            if parents is not None:
                par = parents[lvl - 1]
                nc = int(par.max()) + 1
                P = agglomeration_from_parent(par, nc, nlev)
            else:
                P = agglomeration(nx, ny, nlev)
                nx, ny = nx // 2, ny // 2
                nc = nx * ny
            self.P.append(P)
            self.H.append(sp.csr_matrix(P.T @ self.H[-1] @ P))
            self.ncol.append(nc)
        self.Hz = [column_part(h, n) for h, n in zip(self.H, self.ncol)]
        self.Hz_lu = [spla.splu(h.tocsc()) for h in self.Hz]

    @property
    def nlevels(self):
        return len(self.H)

    def smooth(self, level, x, b, sweeps):
        for _ in range(sweeps):
            x = x + self.omega * self.Hz_lu[level].solve(b - self.H[level] @ x)
        return x

    def vcycle(self, b, level=0):
        x = np.zeros_like(b)
        if level == self.nlevels - 1:
            if self.coarse_cheb is not None:
                lo, hi = self.coarse_cheb
                return chebyshev_solve(lambda v: self.H[level] @ v, self.Hz_lu[level].solve, b,
                                       self.coarse_sweeps, lo, hi)
            return self.smooth(level, x, b, self.coarse_sweeps)
        x = self.smooth(level, x, b, self.pre)
        r = b - self.H[level] @ x
        xc = self.vcycle(self.P[level].T @ r, level + 1)
        x = x + self.P[level] @ xc
        return self.smooth(level, x, b, self.post)


def chebyshev_solve(apply_A, apply_Minv, b, steps, lo, hi):
    """Chebyshev semi-iteration (Golub and Varga, 1961) for A x = b from x = 0, preconditioned by M,
    tuned to eigenvalues of M^-1 A in [lo, hi]; the three-term recurrence of the shifted and scaled
    Chebyshev polynomials (as in Saad, Iterative Methods for Sparse Linear Systems, Alg. 12.1).
    After `steps` preconditioner applications the error is p(M^-1 A) x with
    p(t) = T_steps((theta - t) / delta) / T_steps(theta / delta), theta and delta the centre and
    half-width of the interval."""
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    x_prev = np.zeros_like(b)
    x = apply_Minv(b) / theta
    for _ in range(steps - 1):
        rho_next = 1.0 / (2.0 * sigma - rho)
        x_next = x + rho_next * rho * (x - x_prev) + (2.0 * rho_next / delta) * apply_Minv(b - apply_A(x))
        x_prev, x, rho = x, x_next, rho_next
    return x


def trace_prolongation(mesh: BoxMesh):
    """P: cells -> trace facets, lambda_F = average of the adjacent cells (one sided on lid/ground)."""
    rows = mesh.cell_faces.ravel()
    cols = np.repeat(np.arange(mesh.ncell), 6)
    w = np.where(mesh.boundary[rows], 1.0, 0.5)
    return sp.csr_matrix((w, (rows, cols)), shape=(mesh.ntrace, mesh.ncell))


def line_smoother_matrix(mesh: BoxMesh, S, patch=None):
    """D = blockdiag(S^zz_j) + diag(S^hh): the part of S inverted by LineSmooth.

    patch (optional, one patch index per column): the future-work variant of Sec. 4.2 that caches
    the tridiagonal column matrices over small patches of the grid: every column of a patch uses
    the same S^zz, here the mean of the patch's columns' S^zz entries (below, diagonal, above at
    every level)."""
    Sc = sp.coo_matrix(S)
    zr, zc = Sc.row < mesh.n_zface, Sc.col < mesh.n_zface
    same_col = (Sc.row % mesh.ncol) == (Sc.col % mesh.ncol)
    keep = (zr & zc & same_col) | (~zr & (Sc.row == Sc.col))
    if patch is None:
        return sp.csr_matrix((Sc.data[keep], (Sc.row[keep], Sc.col[keep])), shape=S.shape)
    ncol = mesh.ncol
    patch = np.asarray(patch, np.int64)
    npatch = int(patch.max()) + 1
    count = np.bincount(patch, minlength=npatch).astype(np.float64)
    zz = keep & zr
    rows, cols, vals = Sc.row[zz], Sc.col[zz], Sc.data[zz]
    k, col = rows // ncol, rows % ncol
    off = (cols // ncol) - k + 1  # 0 below, 1 diagonal, 2 above
    mean = np.zeros((3, mesh.nlev + 1, npatch))
    np.add.at(mean, (off, k, patch[col]), vals)
    mean /= count[None, None, :]
    zvals = mean[off, k, patch[col]]
    hh = keep & ~zr
    return sp.csr_matrix((np.concatenate([zvals, Sc.data[hh]]),
                          (np.concatenate([rows, Sc.row[hh]]), np.concatenate([cols, Sc.col[hh]]))), shape=S.shape)


class TwoLevel:
    """Alg. 2 with LineSmooth (Alg. 1) and a pressure multigrid V-cycle coarse solve."""

    def __init__(self, mesh: BoxMesh, S, H, omega=0.6, n_pre=1, n_post=2, mg_levels=4,
                 omega_p=0.9, mg_pre=1, mg_post=2, mg_coarse_sweeps=6, sign=+1.0,
                 mg_coarse_cheb=COARSE_CHEB, coarse=True, smoother_patch=None):
        """coarse=False: no coarse correction, the preconditioner is n_pre + n_post LineSmooth
        sweeps from zero (the paper's hybridised single-level Configuration 2); coarse=("bicgstab",
        rtol): the coarse pressure system solved by BiCGStab preconditioned by the V-cycle to rtol
        (the paper's Configurations 3a and 3b); smoother_patch: a patch index per column, for
        LineSmooth with column matrices cached per patch (``line_smoother_matrix``)."""
        self.mesh, self.S = mesh, sp.csr_matrix(S)
        self.omega, self.n_pre, self.n_post, self.sign = omega, n_pre, n_post, sign
        self.coarse = coarse
        self.D = line_smoother_matrix(mesh, self.S, smoother_patch)
        self.D_lu = spla.splu(self.D.tocsc())
        self.P = trace_prolongation(mesh)
        parents = getattr(mesh, "parents", None)
        self.mg = PressureMultigrid(H, getattr(mesh, "nx", 0), getattr(mesh, "ny", 0), mesh.nlev, mg_levels,
                                    omega_p, mg_pre, mg_post, mg_coarse_sweeps, mg_coarse_cheb,
                                    parents=parents if parents else None)
        ones_c = np.ones(mesh.ncell)
        self.gamma = (H @ ones_c) / (self.P.T @ (self.S @ (self.P @ ones_c)))

    def line_smooth(self, lam, B, sweeps):
        for _ in range(sweeps):
            R = B - self.S @ lam
            lam = lam + self.sign * self.omega * self.D_lu.solve(R)
        return lam

    def __call__(self, B):
        lam = np.zeros_like(B)
        lam = self.line_smooth(lam, B, self.n_pre)
        if not self.coarse:
            return self.line_smooth(lam, B, self.n_post)
        R = B - self.S @ lam
        Bbar = self.gamma * (self.P.T @ R)
        if isinstance(self.coarse, tuple) and self.coarse[0] == "bicgstab":
            from .krylov import bicgstab

            H0 = self.mg.H[0]
            dpi = bicgstab(lambda v: H0 @ v, self.mg.vcycle, Bbar, self.coarse[1])
        else:
            dpi = self.mg.vcycle(Bbar)
        lam = lam + self.P @ dpi
        return self.line_smooth(lam, B, self.n_post)
