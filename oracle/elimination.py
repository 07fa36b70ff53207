"""Elimination of potential temperature and density around the velocity / Exner-pressure solve, and
their back-substitution (test infrastructure).

Follows Sec. 2.1 of the paper (the analytic elimination of theta' from the linearised equations,
which changes the momentum and equation-of-state right-hand sides to
r_u - tau_u dt c_p grad(Pi*) r_theta and r_Pi + r_theta / theta*, the Exner gradient being the
vertical derivative of the projected profile in the discretisation) and Sec. 2.2 (the 3x3 matrix
system in (u, rho, Pi) and the algebraic elimination rho = M3^-1 (R_rho - D u), which turns the
pressure right-hand side into R_Pi + M3^rho M3^-1 R_rho).  After the 2x2 solve, rho' follows from
that same relation and theta' from the theta equation,
theta' = r_theta - tau_theta dt (z_hat . u') d theta*/dz.

Inputs on the mesh of the solver (p = 0): the momentum residual as its broken dual vector
r_u^b(K, F) = <v_F . r_u>_K (as the solver takes it), the density and Exner residuals r_rho, r_Pi
as cell values (W3 fields), the potential temperature residual r_theta as values on the horizontal
facets (the nodes of W_theta, linear in the vertical inside a cell).

Readings taken here (the paper does not spell out these discrete details):

* The linear form of the equation of state uses the same nodal (cell centre) rule as q32,
  m3^rho and m3^Pi, so that R_Pi(K) = w_c (r_Pi + r_theta / theta*) at the centre, w_c the
  one-point weight (the cell volume on the box, det J at the reference centre on the sphere);
  R_rho(K) = <phi r_rho> by the Gauss rule (the exact volume).
* theta' is recovered at each cell's two W_theta nodes (the centres of its bottom and top
  facets) from the cell's own broken velocity, so it is linear in the vertical inside the cell
  and may jump across horizontal facets (d theta*/dz does).  With theta' represented that way
  and the theta equation collocated at those nodes, the algebraic elimination of theta' from
  the discrete four-field system reproduces q22, q32 and the modified right-hand sides exactly
  on the box (``FourFieldSystem``, used by the tests as the monolithic reference).

Parity: pinned by tests against the four-field system solved by sparse LU on tiny boxes (its
solution equals elimination, the 2x2 solve and the back-substitution), against the closed forms
of the right-hand side change on box and cubed-sphere cells, and against invariants (no change
when r_theta = r_rho = 0; theta' = r_theta when theta* is constant; mass conservation of rho').
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .local import rt0_values, volume_rule


def box_map(hx, hy, hz):
    """The cell map of axis-aligned cells with sides (hx, hy, hz) (its origin is irrelevant here)."""
    hx, hy, hz = (np.asarray(a, np.float64) for a in (hx, hy, hz))

    def m(xi, eta, zeta):
        nq = xi.shape[0]
        x = np.stack([np.outer(hx, xi), np.outer(hy, eta), np.outer(hz, zeta)], axis=-1)
        J = np.zeros((hx.shape[0], nq, 3, 3))
        J[:, :, 0, 0] = hx[:, None]
        J[:, :, 1, 1] = hy[:, None]
        J[:, :, 2, 2] = hz[:, None]
        return x + np.array([0.0, 0.0, 1.0]), J  # shifted off the origin; +z is the vertical

    return m


def _geometry(cmap, radial, xi, eta, zeta):
    """Piola-mapped reference RT0 functions, det J, the vertical unit vector and grad(zeta)."""
    x, J = cmap(xi, eta, zeta)
    det = np.linalg.det(J)
    vhat = rt0_values(xi, eta, zeta, np.ones(1), np.ones(1), np.ones(1))[0]  # (nq, 6, 3)
    v = np.einsum("cqde,qae->cqad", J, vhat) / det[:, :, None, None]
    if radial:
        zh = x / np.linalg.norm(x, axis=-1, keepdims=True)
    else:
        zh = np.broadcast_to(np.array([0.0, 0.0, 1.0]), x.shape)
    gzeta = np.linalg.inv(J)[:, :, 2, :]
    return det, v, zh, gzeta


def eliminate_rhs(cmap, radial, fields, consts, r_ub, r_rho, r_thB, r_thT, r_pi):
    """The right-hand sides of the 2x2 system from the residuals of the four-field system.

    cmap, radial: the cell map and the choice of vertical (as for the cell matrices);
    fields: (nc,) arrays thB, thT, piB, piT (theta* and the projected Exner pressure on the bottom
    and top facets), rhoc; consts: dt, tau_u, cp.  r_ub (nc, 6); r_rho, r_pi, r_thB, r_thT (nc,).
    Returns (r_ub_bar (nc, 6), r_pi_bar (nc,)): the broken momentum dual vector of
    r_u - tau_u dt c_p z_hat dPi*/dz r_theta (Sec. 2.1) and R_Pi + M3^rho M3^-1 R_rho (Sec. 2.2).
    """
    dt, tu, cp = consts["dt"], consts["tau_u"], consts["cp"]
    thB, thT, piB, piT, rhoc = (fields[k] for k in ("thB", "thT", "piB", "piT", "rhoc"))
    qx, qy, qz, qw = volume_rule()
    det, v, zh, gz = _geometry(cmap, radial, qx, qy, qz)
    wq = qw[None, :] * det
    dzpi = np.einsum("cqd,cqd->cq", zh, (piT - piB)[:, None, None] * gz)
    rth_q = r_thB[:, None] * (1.0 - qz)[None, :] + r_thT[:, None] * qz[None, :]
    vz = np.einsum("cqad,cqd->cqa", v, zh)
    # <v_F . (-tau_u dt c_p z_hat dPi*/dz r_theta)>_K
    r_ub_bar = r_ub - tu * dt * cp * np.einsum("cq,cqa->ca", wq * dzpi * rth_q, vz)
    # R_rho = <phi r_rho> (Gauss), M3 = <phi phi>, M3^rho and R_Pi by the one-point centre rule
    m3 = wq.sum(axis=1)
    h = np.array([0.5])
    detc = _geometry(cmap, radial, h, h, h)[0][:, 0]
    thc, rthc = 0.5 * (thB + thT), 0.5 * (r_thB + r_thT)
    R_pi = detc * (r_pi + rthc / thc)
    R_rho = m3 * r_rho
    m3rho = detc / rhoc
    return r_ub_bar, R_pi + m3rho / m3 * R_rho


def back_substitute(cmap, radial, fields, consts, r_rho, r_thB, r_thT, u_b):
    """rho' and theta' from the velocity of the 2x2 solve.

    u_b (nc, 6): each cell's outward fluxes (the recovered broken velocity).  Returns
    (rho (nc,), theta (nc, 2)): rho' = M3^-1 (R_rho - D u) with D(phi, u) =
    tau_rho dt <phi div(rho* u)> (Sec. 2.2), and theta' = r_theta - tau_theta dt (z_hat . u) dtheta*/dz
    at the cell's bottom and top W_theta nodes (Sec. 2.1).
    """
    dt, tr, tt = consts["dt"], consts["tau_rho"], consts["tau_theta"]
    thB, thT, rhoc = fields["thB"], fields["thT"], fields["rhoc"]
    qx, qy, qz, qw = volume_rule()
    det, v, zh, gz = _geometry(cmap, radial, qx, qy, qz)
    wq = qw[None, :] * det
    m3 = wq.sum(axis=1)
    # div v_F = 1 / det J for every F (unit outward flux of the reference functions)
    dD = tr * dt * rhoc[:, None] * np.einsum("cq,cq->c", wq, 1.0 / det)[:, None] * np.ones((1, 6))
    rho = (m3 * r_rho - np.einsum("ca,ca->c", dD, u_b)) / m3
    theta = np.zeros((u_b.shape[0], 2))
    for e, (zeta, rth) in enumerate(((0.0, r_thB), (1.0, r_thT))):
        h = np.array([0.5])
        d_e, v_e, zh_e, gz_e = _geometry(cmap, radial, h, h, np.array([zeta]))
        uz = np.einsum("cad,cd,ca->c", v_e[:, 0], zh_e[:, 0], u_b)
        dzth = (thT - thB) * np.einsum("cd,cd->c", zh_e[:, 0], gz_e[:, 0])
        theta[:, e] = rth - tt * dt * uz * dzth
    return rho, theta


class FourFieldSystem:
    """The linear system in (u, rho, theta', Pi) before any elimination, on a periodic box.

    Velocity in the continuous W2 (global orientation, no dof on the lid and ground), rho and Pi
    cell constants, theta' two values per cell (its bottom and top W_theta nodes, linear in the
    vertical between them).  Rows:
      momentum  m2(w, u) + tau_u dt c_p <(z.w) theta' dPi*/dz> + g(w, Pi) = <w . r_u>
      density   d(phi, u) + m3(phi, rho) = <phi r_rho>
      theta     theta'(x_e) + tau_theta dt (z.u)(x_e) dtheta*/dz = r_theta(x_e) at both nodes x_e
      state     (1-kappa)/kappa <psi Pi / Pi*> - <psi rho / rho*> - <psi theta' / theta*> = <psi r_Pi>
    with the Gauss rule for m2, g, d, m3 and the momentum term, the centre rule for the state row
    (Sec. 2.1, 2.2).  Eliminating theta' and then rho gives the 2x2 system of Sec. 2.2.
    """

    def __init__(self, mesh, prob, loc):
        from .mixed import MixedSystem

        self.mesh = mesh
        self.mixed = MixedSystem(mesh, loc, prob)
        mx = self.mixed
        nc = mesh.ncell
        k = mesh.cell_layer
        col = mesh.cell_iy * mesh.nx + mesh.cell_ix
        hx, hy, hz = np.full(nc, mesh.dx), np.full(nc, mesh.dy), mesh.dz[k]
        thB, thT = prob.theta_w[k, col], prob.theta_w[k + 1, col]
        piB, piT = prob.exner_hat_w[k, col], prob.exner_hat_w[k + 1, col]
        rhoc, pic = prob.rho_c[k, col], prob.exner_c[k, col]
        dt, tu, tr, tt, cp, kappa = prob.dt, prob.tau_u, prob.tau_rho, prob.tau_theta, prob.cp, prob.kappa
        qx, qy, qz, qw = volume_rule()
        v = rt0_values(qx, qy, qz, hx, hy, hz)
        vol = hx * hy * hz
        wq = qw[None, :] * vol[:, None]
        dzpi, dzth = (piT - piB) / hz, (thT - thB) / hz
        # momentum-theta coupling per cell: C[c, a, e] = tau_u dt c_p <(z.v_a) phi_e dPi*/dz>
        phi = np.stack([1.0 - qz, qz], axis=1)  # (nq, 2) linear nodal functions in the vertical
        Ccell = tu * dt * cp * np.einsum("cq,cqa,qe->cae", wq * dzpi[:, None], v[:, :, :, 2], phi)
        # theta rows: (z.u)(x_e) for u = v_a at the bottom / top node (facet centre)
        vn = np.stack([rt0_values(np.array([0.5]), np.array([0.5]), np.array([z]), hx, hy, hz)[:, 0, :, 2]
                       for z in (0.0, 1.0)], axis=1)  # (nc, 2, 6)
        Bcell = tt * dt * dzth[:, None, None] * vn
        nu, npr = mx.nu, nc
        ith = lambda c, e: 2 * c + e  # noqa: E731
        rows, cols, vals = [], [], []

        def add(r, c_, x):
            rows.append(np.asarray(r).ravel())
            cols.append(np.asarray(c_).ravel())
            vals.append(np.asarray(x, np.float64).ravel())

        # blocks: u [0, nu), rho [nu, nu + nc), theta [nu + nc, nu + 3 nc), Pi [nu + 3 nc, nu + 4 nc)
        o_r, o_t, o_p = nu, nu + nc, nu + 3 * nc
        cells = np.arange(nc)
        # velocity block without q22: m2 (no Coriolis on the box) in global orientation
        cf, cs = mesh.cell_faces, mesh.cell_sign
        for a in range(6):
            ua = mx.udof[cf[:, a]]
            oka = ua >= 0
            for b in range(6):
                ub = mx.udof[cf[:, b]]
                ok = oka & (ub >= 0)
                add(ua[ok], ub[ok], (cs[:, a] * cs[:, b] * loc["m2"][:, a, b])[ok])
            for e in range(2):
                add(ua[oka], o_t + ith(cells, e)[oka], (cs[:, a] * Ccell[:, a, e])[oka])
                add(o_t + ith(cells, e)[oka], ua[oka], (cs[:, a] * Bcell[:, e, a])[oka])
            # density row: d(phi, v_a) = tau_rho dt rho* (unit flux); Pi column: g (no facet term here)
            add(o_r + cells[oka], ua[oka], (cs[:, a] * tr * dt * rhoc)[oka])
        G = sp.coo_matrix(mx.G)
        add(G.row, o_p + G.col, G.data)
        add(o_r + cells, o_r + cells, vol)  # m3
        for e in range(2):
            add(o_t + ith(cells, e), o_t + ith(cells, e), np.ones(nc))
        # state row at the centre: theta'(c) = (theta'_B + theta'_T) / 2
        thc = 0.5 * (thB + thT)
        add(o_p + cells, o_p + cells, (1 - kappa) / kappa * vol / pic)
        add(o_p + cells, o_r + cells, -vol / rhoc)
        for e in range(2):
            add(o_p + cells, o_t + ith(cells, e), -0.5 * vol / thc)
        cat = np.concatenate
        n = nu + 4 * nc
        self.matrix = sp.csc_matrix((cat(vals), (cat(rows), cat(cols))), shape=(n, n))
        self.offsets = (o_r, o_t, o_p)
        self.vol = vol

    def solve(self, r_ub, r_rho, r_thB, r_thT, r_pi):
        """Returns (u (nu,), rho (nc,), theta (nc, 2), Pi (nc,)) for cell-ordered residuals."""
        mx, nc = self.mixed, self.mesh.ncell
        Ru = mx.rhs(r_ub, np.zeros(nc))[: mx.nu]
        rhs = np.concatenate([Ru, self.vol * r_rho, np.stack([r_thB, r_thT], axis=1).ravel(), self.vol * r_pi])
        sol = spla.splu(self.matrix).solve(rhs)
        o_r, o_t, o_p = self.offsets
        return sol[:o_r], sol[o_r:o_t], sol[o_t:o_p].reshape(nc, 2), sol[o_p:]
