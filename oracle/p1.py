"""Next-to-lowest-order (p = 1) hybridised system on the box (test infrastructure, FP64).

The paper states the method for general order p (Sec. 2.2: W2 = RT_p, W3 = Q_p^DG, Gauss rules
with n = p + 3 points per direction, q32, m3^rho and m3^Pi at the nodal points of W3; Sec. 2.4:
broken velocity, trace space of degree p per facet) and gives the local sizes for p = 1 in its
table of unknowns (44 x 44 mixed, 24 x 24 hybridised).  This module writes that out for p = 1:

  - velocity: broken RT1 = Q(2,1,1) x Q(1,2,1) x Q(1,1,2), 36 functions per cell.  Each component
    is a Lagrange function on the nodes {0, 1/2, 1} in its own direction and on the two Gauss
    points in the other two.  Dofs: on each face the outward normal component at the 2 x 2 face
    Gauss points (24, face f dof i = 4 f + i), then the interior values at the mid-plane nodes (12).
  - pressure: DG1 = Q1, nodal at the 2 x 2 x 2 Gauss points (8), so the W3 mass matrix is diagonal
    and the nodal rule is the Gauss rule.
  - trace: Q1 on each facet, nodal at the 2 x 2 face Gauss points (4 per facet, global index
    4 F + i), so C_K and K_K are diagonal on the face dofs.
  - theta* and the projected Exner pressure: linear in the vertical in each cell, given by their
    values on the bottom and top facets (as for p = 0).

Face order W, E, S, N, B, T (outward normals -x, +x, -y, +y, -z, +z); tangential coordinates of a
face: (y, z) for x-faces, (x, z) for y-faces, (x, y) for z-faces; face point i = 2 t1 + t2.

Parity: pinned (tests) by the nodal identities of the bases, the divergence theorem per basis
function, exactness of the n = 4 rule (n = 6 gives the same matrices), the RT0 and DG0 fields
embedded in RT1 and DG1 reproducing the p = 0 cell matrices of every form but the nodal q32
(which is checked against its own definition), the table of unknowns, a dense brute-force solve
of the hybridised system on tiny meshes, the equivalence with the continuous-RT1 mixed system,
continuity of the recovered normal velocity and symmetry / definiteness of S in the symmetric case.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .local import cell_data
from .mesh import BoxMesh

NU, NP, NF = 36, 8, 24  # velocity, pressure, face (trace) dofs per cell
NX = NU + NP
G2 = 0.5 + np.array([-0.5, 0.5]) / np.sqrt(3.0)  # 2-point Gauss nodes on [0, 1]
Q3 = np.array([0.0, 0.5, 1.0])
FACE_DIR = [0, 0, 1, 1, 2, 2]
FACE_SIGN = [-1.0, 1.0, -1.0, 1.0, -1.0, 1.0]
TANG = {0: (1, 2), 1: (0, 2), 2: (0, 1)}  # tangential directions of a face / interior family


def gauss(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def lag(nodes, j, x):
    """Lagrange polynomial j on ``nodes`` and its derivative at points x."""
    v = np.ones_like(x)
    for m, xm in enumerate(nodes):
        if m != j:
            v = v * (x - xm) / (nodes[j] - xm)
    d = np.zeros_like(x)
    for m, xm in enumerate(nodes):
        if m == j:
            continue
        t = np.ones_like(x) / (nodes[j] - xm)
        for q, xq in enumerate(nodes):
            if q not in (j, m):
                t = t * (x - xq) / (nodes[j] - xq)
        d = d + t
    return v, d


def rt1_table():
    """(direction d, normal node a, tangential Gauss indices (t1, t2), sign) for the 36 functions."""
    out = []
    for f in range(6):
        d = FACE_DIR[f]
        a = 0 if FACE_SIGN[f] < 0 else 2
        for i in range(4):
            out.append((d, a, (i // 2, i % 2), FACE_SIGN[f]))
    for d in range(3):
        for i in range(4):
            out.append((d, 1, (i // 2, i % 2), 1.0))
    return out


RT1 = rt1_table()


def rt1_values(p, h):
    """Values (nc, nq, 36, 3) and divergences (nc, nq, 36) at reference points p = (x, y, z)."""
    hx, hy, hz = h
    nc, nq = hx.shape[0], p[0].shape[0]
    val = np.zeros((nq, NU, 3))
    dv = np.zeros((nq, NU, 3))  # d/d(reference coordinate of the own direction)
    for j, (d, a, (t1, t2), sgn) in enumerate(RT1):
        ln, dln = lag(Q3, a, p[d])
        u, v = TANG[d]
        g1, _ = lag(G2, t1, p[u])
        g2, _ = lag(G2, t2, p[v])
        val[:, j, d] = sgn * ln * g1 * g2
        dv[:, j, d] = sgn * dln * g1 * g2
    hs = np.stack([hx, hy, hz], axis=1)  # (nc, 3)
    vals = np.broadcast_to(val[None], (nc, nq, NU, 3)).copy()
    div = np.einsum("qjd,cd->cqj", dv, 1.0 / hs)
    return vals, div


def dg1_values(p):
    """Values (nq, 8) of the Q1 functions nodal at the 2x2x2 Gauss points; index 4 i + 2 j + k."""
    out = np.zeros((p[0].shape[0], NP))
    for i in range(2):
        for j in range(2):
            for k in range(2):
                out[:, 4 * i + 2 * j + k] = lag(G2, i, p[0])[0] * lag(G2, j, p[1])[0] * lag(G2, k, p[2])[0]
    return out


def volume_rule(n):
    x, w = gauss(n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    W = w[:, None, None] * w[None, :, None] * w[None, None, :]
    return (X.ravel(), Y.ravel(), Z.ravel()), W.ravel()


def face_points(f, n):
    """Reference points (3 arrays) and weights (summing to 1) of the n x n rule on face f, ordered
    with the first tangential coordinate slowest."""
    x, w = gauss(n)
    T1, T2 = np.meshgrid(x, x, indexing="ij")
    d = FACE_DIR[f]
    u, v = TANG[d]
    p = [None, None, None]
    p[d] = np.full(T1.size, 0.0 if FACE_SIGN[f] < 0 else 1.0)
    p[u], p[v] = T1.ravel(), T2.ravel()
    return tuple(p), (w[:, None] * w[None, :]).ravel()


def local_matrices(mesh: BoxMesh, prob, n_quad: int = 4, cells=None):
    """A (nc, 44, 44) = [[M2 - Q22, G^b], [Q32 + M3rho M3^-1 D, M3Pi]], K and C (nc, 36, 24), and the
    separate forms, for every cell (Sec. 2.2 forms with the n-point rule; nodal rule for q32,
    m3^rho, m3^Pi)."""
    cd = cell_data(mesh, prob, cells)
    dt, tu, tr, tt, cp, kappa = prob.dt, prob.tau_u, prob.tau_rho, prob.tau_theta, prob.cp, prob.kappa
    hx, hy, hz = cd["hx"], cd["hy"], cd["hz"]
    vol = hx * hy * hz
    thB, thT, piB, piT, pic, rhoc = cd["thB"], cd["thT"], cd["piB"], cd["piT"], cd["pic"], cd["rhoc"]
    dth, dpi = (thT - thB) / hz, (piT - piB) / hz
    nc = hx.shape[0]
    pq, wq0 = volume_rule(n_quad)
    v, div = rt1_values(pq, (hx, hy, hz))
    phi = dg1_values(pq)  # (nq, 8)
    wq = wq0[None, :] * vol[:, None]
    theta_q = thB[:, None] * (1.0 - pq[2])[None, :] + thT[:, None] * pq[2][None, :]
    m2 = np.einsum("cq,cqad,cqbd->cab", wq, v, v)
    q22 = tu * tt * dt * dt * cp * np.einsum("cq,cqa,cqb->cab", wq * (dpi * dth)[:, None], v[..., 2], v[..., 2])
    divthw = theta_q[:, :, None] * div + v[..., 2] * dth[:, None, None]
    gb = -tu * dt * cp * np.einsum("cq,cqa,qp->cap", wq, divthw, phi)
    dD = tr * dt * rhoc[:, None, None] * np.einsum("cq,qp,cqa->cpa", wq, phi, div)
    m3 = np.einsum("cq,qp,qr->cpr", wq, phi, phi)
    # nodal rule of W3: the 2x2x2 Gauss points, weight vol / 8 each
    pn, wn0 = volume_rule(2)
    vn, _ = rt1_values(pn, (hx, hy, hz))
    phin = dg1_values(pn)  # identity up to ordering
    wn = wn0[None, :] * vol[:, None]
    theta_n = thB[:, None] * (1.0 - pn[2])[None, :] + thT[:, None] * pn[2][None, :]
    q32 = tt * dt * np.einsum("cq,qp,cqa->cpa", wn * dth[:, None] / theta_n, phin, vn[..., 2])
    m3rho = np.einsum("cq,qp,qr->cpr", wn / rhoc[:, None], phin, phin)
    m3pi = (1.0 - kappa) / kappa * np.einsum("cq,qp,qr->cpr", wn / pic[:, None], phin, phin)
    K = np.zeros((nc, NU, NF))
    C = np.zeros((nc, NU, NF))
    area = np.stack([hy * hz, hy * hz, hx * hz, hx * hz, hx * hy, hx * hy], axis=1)
    for f in range(6):
        pf, wf0 = face_points(f, n_quad)
        vf, _ = rt1_values(pf, (hx, hy, hz))
        vnorm = FACE_SIGN[f] * vf[..., FACE_DIR[f]]  # outward normal component (nc, nqf, 36)
        u, w_ = TANG[FACE_DIR[f]]
        nu = np.stack([lag(G2, i // 2, pf[u])[0] * lag(G2, i % 2, pf[w_])[0] for i in range(4)], axis=1)
        th_f = thB[:, None] * (1.0 - pf[2])[None, :] + thT[:, None] * pf[2][None, :]
        wf = wf0[None, :] * area[:, f][:, None]
        C[:, :, 4 * f: 4 * f + 4] = np.einsum("cq,cqa,qi->cai", wf, vnorm, nu)
        K[:, :, 4 * f: 4 * f + 4] = tu * dt * cp * np.einsum("cq,cq,cqa,qi->cai", wf, th_f, vnorm, nu)
    drow = q32 + np.einsum("cpq,cqr,cra->cpa", m3rho, np.linalg.inv(m3), dD)
    A = np.zeros((nc, NX, NX))
    A[:, :NU, :NU] = m2 - q22
    A[:, :NU, NU:] = gb
    A[:, NU:, :NU] = drow
    A[:, NU:, NU:] = m3pi
    return dict(A=A, K=K, C=C, m2=m2, q22=q22, gb=gb, d=dD, m3=m3, q32=q32, m3rho=m3rho, m3pi=m3pi)


def cell_dofs(mesh: BoxMesh):
    """Global trace dof of each local face dof: (ncell, 24) = 4 F + i."""
    cf = mesh.cell_faces
    return (4 * cf[:, :, None] + np.arange(4)[None, None, :]).reshape(mesh.ncell, NF)


def cell_trace_operator(loc):
    """S_K = C_K^T [A_K^-1 [K_K; 0]]_u (24 x 24 per cell)."""
    n = loc["A"].shape[0]
    Kh = np.zeros((n, NX, NF))
    Kh[:, :NU, :] = loc["K"]
    X = np.linalg.solve(loc["A"], Kh)
    return np.einsum("caf,cag->cfg", loc["C"], X[:, :NU, :])


class HybridP1:
    """S lambda = B_lambda on 4 trace dofs per facet, recovery, and the dense KKT brute force."""

    def __init__(self, mesh: BoxMesh, loc: dict):
        self.mesh, self.loc = mesh, loc
        self.ntrace = 4 * mesh.ntrace
        self.dofs = cell_dofs(mesh)
        self.S_cell = cell_trace_operator(loc)
        rows = np.repeat(self.dofs[:, :, None], NF, axis=2).ravel()
        cols = np.repeat(self.dofs[:, None, :], NF, axis=1).ravel()
        self.S = sp.csr_matrix((self.S_cell.ravel(), (rows, cols)), shape=(self.ntrace, self.ntrace))
        self.S.sum_duplicates()

    def rhs(self, r_u, r_p):
        """r_u (ncell, 36), r_p (ncell, 8) -> B_lambda = C^T A^-1 R."""
        R = np.concatenate([r_u, r_p], axis=1)
        X = np.linalg.solve(self.loc["A"], R[:, :, None])[:, :, 0]
        b = np.einsum("caf,ca->cf", self.loc["C"], X[:, :NU])
        B = np.zeros(self.ntrace)
        np.add.at(B, self.dofs.ravel(), b.ravel())
        return B

    def recover(self, lam, r_u, r_p):
        R = np.concatenate([r_u, r_p], axis=1)
        R[:, :NU] -= np.einsum("caf,cf->ca", self.loc["K"], lam[self.dofs])
        X = np.linalg.solve(self.loc["A"], R[:, :, None])[:, :, 0]
        return X[:, :NU], X[:, NU:]

    def solve_direct(self, r_u, r_p):
        B = self.rhs(r_u, r_p)
        lam = spla.splu(self.S.tocsc()).solve(B)
        u, p = self.recover(lam, r_u, r_p)
        return lam, u, p, B

    def solve_kkt_dense(self, r_u, r_p):
        n = self.mesh.ncell
        N = NX * n + self.ntrace
        M = np.zeros((N, N))
        for c in range(n):
            M[NX * c: NX * c + NX, NX * c: NX * c + NX] = self.loc["A"][c]
            for a in range(NU):
                for f in range(NF):
                    F = NX * n + self.dofs[c, f]
                    M[NX * c + a, F] += self.loc["K"][c, a, f]
                    M[F, NX * c + a] += self.loc["C"][c, a, f]
        rhs = np.zeros(N)
        rhs[: NX * n] = np.concatenate([r_u, r_p], axis=1).ravel()
        sol = np.linalg.solve(M, rhs)
        X = sol[: NX * n].reshape(n, NX)
        return sol[NX * n:], X[:, :NU], X[:, NU:]


class MixedP1:
    """The unhybridised system in continuous RT1: one velocity dof per face point of every interior
    facet (global orientation +x, +y, +z), the 12 interior dofs of every cell, no dofs on the
    lid and ground.  Assembled from the cell matrices by the sign map; valid as stated when theta*
    is single valued on every facet (then the facet term of g vanishes)."""

    def __init__(self, mesh: BoxMesh, loc: dict):
        self.mesh = mesh
        nf = mesh.ntrace
        interior = ~mesh.boundary
        fdof = -np.ones(nf, np.int64)
        fdof[interior] = np.arange(int(interior.sum()))
        nfi = int(interior.sum())
        self.nu = 4 * nfi + 12 * mesh.ncell
        self.np_ = NP * mesh.ncell
        n = mesh.ncell
        gmap = np.zeros((n, NU), np.int64)
        sign = np.zeros((n, NU))
        for f in range(6):
            F = fdof[mesh.cell_faces[:, f]]
            for i in range(4):
                gmap[:, 4 * f + i] = np.where(F >= 0, 4 * F + i, -1)
                sign[:, 4 * f + i] = np.where(F >= 0, mesh.cell_sign[:, f], 0.0)
        gmap[:, NF:] = 4 * nfi + 12 * np.arange(n)[:, None] + np.arange(12)[None, :]
        sign[:, NF:] = 1.0
        pmap = self.nu + NP * np.arange(n)[:, None] + np.arange(NP)[None, :]
        full = np.concatenate([gmap, pmap], axis=1)
        fsign = np.concatenate([sign, np.ones((n, NP))], axis=1)
        ok = full >= 0
        rows = np.repeat(full[:, :, None], NX, axis=2)
        cols = np.repeat(full[:, None, :], NX, axis=1)
        vals = fsign[:, :, None] * fsign[:, None, :] * loc["A"]
        keep = ok[:, :, None] & ok[:, None, :]
        N = self.nu + self.np_
        self.matrix = sp.csc_matrix((vals[keep], (rows[keep], cols[keep])), shape=(N, N))
        self.full, self.fsign = full, fsign

    def rhs(self, r_u, r_p):
        R = np.concatenate([r_u, r_p], axis=1)
        out = np.zeros(self.nu + self.np_)
        ok = self.full >= 0
        np.add.at(out, self.full[ok], (self.fsign * R)[ok])
        return out

    def solve(self, r_u, r_p):
        sol = spla.splu(self.matrix).solve(self.rhs(r_u, r_p))
        return sol

    def broken(self, sol):
        """Broken (outward) velocity (ncell, 36) and pressure (ncell, 8) of a mixed solution."""
        x = np.where(self.full >= 0, sol[np.maximum(self.full, 0)], 0.0) * self.fsign
        return x[:, :NU], x[:, NU:]


# ---- the two-level preconditioner at order 1 (Alg. 1 and Alg. 2 with the DG0 coarse space) ----

def trace_prolongation(mesh: BoxMesh):
    """P: DG0 cells -> order-1 trace, every dof of a facet = the average of its two cells (its one
    cell on the lid and the ground)."""
    rows, cols, vals = [], [], []
    cf = mesh.cell_faces
    for f in range(6):
        F = cf[:, f]
        w = np.where(mesh.boundary[F], 1.0, 0.5)
        for i in range(4):
            rows.append(4 * F + i)
            cols.append(np.arange(mesh.ncell))
            vals.append(w)
    cat = np.concatenate
    return sp.csr_matrix((cat(vals), (cat(rows), cat(cols))), shape=(4 * mesh.ntrace, mesh.ncell))


def line_smoother_matrix(mesh: BoxMesh, S):
    """D of LineSmooth at order 1: S restricted to the couplings between dofs of horizontal facets
    of the same column (block tridiagonal with 4x4 blocks), and the diagonal of S on the dofs of
    vertical facets (point Jacobi)."""
    S = sp.coo_matrix(S)
    nz = mesh.n_zface
    Fr, Fc = S.row // 4, S.col // 4
    zr, zc = Fr < nz, Fc < nz
    same_col = zr & zc & ((Fr % mesh.ncol) == (Fc % mesh.ncol))
    keep = same_col | (~zr & (S.row == S.col))
    return sp.csr_matrix((S.data[keep], (S.row[keep], S.col[keep])), shape=S.shape)


class TwoLevelP1:
    """Alg. 2 at order 1: LineSmooth (n_pre) from zero, residual, B = Gamma P^T R, one pressure
    multigrid V-cycle on the order-0 H of the same mesh, lambda += P dPi, LineSmooth (n_post)."""

    def __init__(self, mesh: BoxMesh, S, H, omega=0.6, n_pre=1, n_post=2, mg_levels=4, omega_p=0.9, mg_pre=1,
                 mg_post=2, mg_coarse_sweeps=6, mg_coarse_cheb=(0.02, 2.0), coarse=True):
        from .precond import PressureMultigrid

        self.mesh, self.S = mesh, sp.csr_matrix(S)
        self.omega, self.n_pre, self.n_post, self.coarse = omega, n_pre, n_post, coarse
        self.D = line_smoother_matrix(mesh, self.S)
        self.D_lu = spla.splu(self.D.tocsc())
        self.P = trace_prolongation(mesh)
        self.mg = PressureMultigrid(H, mesh.nx, mesh.ny, mesh.nlev, mg_levels, omega_p, mg_pre, mg_post,
                                    mg_coarse_sweeps, mg_coarse_cheb)
        ones = np.ones(mesh.ncell)
        self.gamma = (H @ ones) / (self.P.T @ (self.S @ (self.P @ ones)))

    def line_smooth(self, lam, B, sweeps):
        for _ in range(sweeps):
            lam = lam + self.omega * self.D_lu.solve(B - self.S @ lam)
        return lam

    def __call__(self, B):
        lam = self.line_smooth(np.zeros_like(B), B, self.n_pre)
        if not self.coarse:  # LineSmooth alone (the single-level configuration)
            return self.line_smooth(lam, B, self.n_post)
        dpi = self.mg.vcycle(self.gamma * (self.P.T @ (B - self.S @ lam)))
        return self.line_smooth(lam + self.P @ dpi, B, self.n_post)
