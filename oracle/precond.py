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

Coarse-space devices (measurements, not part of the path): the conforming
vertex (Q1) coarse space that Sec. 4.2 names, read as the trilinear function on
the hexahedral box whose facet value is its mean over the facet; the
agglomerated cell spaces of the multigrid levels; Alg. 2 with an exact Galerkin
coarse solve; and the best correction in a space after a given cycle.

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


def vertex_trace_prolongation(mesh: BoxMesh):
    """P_v: vertex values -> trace facets, lambda_F = the mean over F of the trilinear (Q1)
    function with those vertex values, i.e. the average of the facet's four corners.

    The conforming piecewise linear coarse space that Sec. 4.2 names as an alternative to the
    piecewise constant one, in its tensor-product form on the extruded hexahedral box: one value per
    vertex, vertex (k, ix, iy) at height z[k] on the south-west corner of column (ix, iy), numbered
    k * ncol + iy * nx + ix (periodic in x and y, levels 0..L)."""
    L, nx, ny, ncol = mesh.nlev, mesh.nx, mesh.ny, mesh.ncol

    def vert(k, ix, iy):
        return k * ncol + (iy % ny) * nx + (ix % nx)

    k = np.arange(L + 1)[:, None, None]
    iy = np.arange(ny)[None, :, None]
    ix = np.arange(nx)[None, None, :]
    rows, cols = [], []
    zf = np.broadcast_to(mesh.zface(k, ix, iy), (L + 1, ny, nx))
    for a, b in ((0, 0), (1, 0), (0, 1), (1, 1)):
        rows.append(zf.ravel())
        cols.append(np.broadcast_to(vert(k, ix + a, iy + b), zf.shape).ravel())
    k = k[:-1]
    xf = np.broadcast_to(mesh.xface(k, ix, iy), (L, ny, nx))
    yf = np.broadcast_to(mesh.yface(k, ix, iy), (L, ny, nx))
    for dk in (0, 1):
        for b in (0, 1):  # the west facet spans the corners (ix, iy) and (ix, iy + 1)
            rows.append(xf.ravel())
            cols.append(np.broadcast_to(vert(k + dk, ix, iy + b), xf.shape).ravel())
        for a in (0, 1):  # the south facet spans the corners (ix, iy) and (ix + 1, iy)
            rows.append(yf.ravel())
            cols.append(np.broadcast_to(vert(k + dk, ix + a, iy), yf.shape).ravel())
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    return sp.csr_matrix((np.full(rows.size, 0.25), (rows, cols)), shape=(mesh.ntrace, ncol * (L + 1)))


def agglomerated_cell_injection(mesh: BoxMesh, parents):
    """Q_l: cells of the 2^l x 2^l agglomerated level -> fine cells (injection), for the parent maps
    of the horizontal agglomeration (one per level below the finest); no vertical coarsening."""
    cols = np.arange(mesh.ncol)
    for par in parents:
        cols = np.asarray(par)[cols]
    ncl = int(cols.max()) + 1
    rows = np.arange(mesh.ncell)
    return sp.csr_matrix((np.ones(rows.size), (rows, (rows // mesh.ncol) * ncl + cols[rows % mesh.ncol])),
                         shape=(mesh.ncell, mesh.nlev * ncl))


class GalerkinTwoLevel:
    """Alg. 2 with LineSmooth (Alg. 1) as in ``TwoLevel``, the coarse space given by its
    prolongation P_c to the trace space and the coarse system solved exactly: after the
    pre-smoothing, lambda += P_c (P_c^T S P_c)^-1 P_c^T (B - S lambda).  With P_c = P (the DG0
    space) this is the best correction that space admits; with ``vertex_trace_prolongation`` it is
    the conforming coarse space of Sec. 4.2.  A measuring device for what a coarse space could
    give at best, not a method to run at scale (a sparse LU of the coarse system)."""

    def __init__(self, smoother: TwoLevel, Pc):
        self.sm = smoother
        self.Pc = sp.csr_matrix(Pc)
        self.A = (self.Pc.T @ smoother.S @ self.Pc).tocsc()
        self.lu = spla.splu(self.A)

    def __call__(self, B):
        sm = self.sm
        lam = sm.line_smooth(np.zeros_like(B), B, sm.n_pre)
        R = B - sm.S @ lam
        lam = lam + self.Pc @ self.lu.solve(self.Pc.T @ R)
        return sm.line_smooth(lam, B, sm.n_post)


class BestCorrectionAfter:
    """The best correction in a coarse space after a preconditioner M: z = M(B), then
    z += P_c (P_c^T S P_c)^-1 P_c^T (B - S z).  The upper bound on what any correction stage
    placed after the coarse correction of Alg. 2 can do with its output confined to the range of
    P_c (the S-orthogonal projection of the remaining error onto that range)."""

    def __init__(self, M, S, Pc):
        self.M, self.S = M, sp.csr_matrix(S)
        self.Pc = sp.csr_matrix(Pc)
        self.lu = spla.splu((self.Pc.T @ self.S @ self.Pc).tocsc())

    def __call__(self, B):
        z = self.M(B)
        return z + self.Pc @ self.lu.solve(self.Pc.T @ (B - self.S @ z))
