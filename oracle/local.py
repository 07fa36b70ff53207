"""Cell matrices of the lowest-order (p = 0) hybridised system, by quadrature.

Test infrastructure (oracle).  Follows Sec. 2.2 of the paper (weak form and
the eight bilinear forms; Gauss quadrature with n = p + 3 points per
direction; q32, m3^rho and m3^Pi at the W3 nodal point, i.e. the cell centre
for p = 0) and Sec. 2.4 (broken space, forms g^b, k and c).

Basis: broken lowest-order Raviart-Thomas functions on an axis-aligned cell,
one per face, scaled to unit outward flux through their own face (so the
velocity dof is that flux).  Potential temperature and the projected Exner
pressure live in the vertically continuous space W_theta: linear in the
vertical inside a cell, given by their values on the bottom and top facets.
W3 functions are cell constants; the trace space holds one constant per
facet.

Readings of the paper taken here: the mu term of the velocity mass form is a
damping rate that is zero (its printed definition duplicates q22 and is not
dimensionally consistent); Omega = 0 on the box; tau_u, tau_rho, tau_theta
given by the input.

Parity: pinned by tests against the closed forms of the p = 0 box cell
matrices derived by hand (mass blocks a_x m, a_y m, (1 + beta) a_z m; g and k
from the divergence theorem; d = tau_rho dt with the buoyancy correction on
B/T), against the exact flux/divergence identities of the basis, and the
local sizes of the paper's table of unknowns (7x7 mixed, 6x6 hybridised).
"""

from __future__ import annotations

import numpy as np

from .mesh import BoxMesh

_GX, _GW = np.polynomial.legendre.leggauss(3)
GAUSS_X = 0.5 * (_GX + 1.0)
GAUSS_W = 0.5 * _GW

# local face order and outward normals
FACE_NORMALS = np.array(
    [[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]], np.float64
)


def rt0_values(xi, eta, zeta, hx, hy, hz):
    """Values of the six broken RT0 basis functions at reference points.

    xi, eta, zeta: arrays of shape (nq,); hx, hy, hz: arrays of shape (nc,).
    Returns an array (nc, nq, 6, 3).
    """
    nc, nq = hx.shape[0], xi.shape[0]
    v = np.zeros((nc, nq, 6, 3))
    ayz = (1.0 / (hy * hz))[:, None]
    axz = (1.0 / (hx * hz))[:, None]
    axy = (1.0 / (hx * hy))[:, None]
    v[:, :, 0, 0] = -(1.0 - xi)[None, :] * ayz
    v[:, :, 1, 0] = xi[None, :] * ayz
    v[:, :, 2, 1] = -(1.0 - eta)[None, :] * axz
    v[:, :, 3, 1] = eta[None, :] * axz
    v[:, :, 4, 2] = -(1.0 - zeta)[None, :] * axy
    v[:, :, 5, 2] = zeta[None, :] * axy
    return v


def rt0_div(hx, hy, hz):
    """Divergence of each basis function: d/dx of the x-component etc. -> (nc, 6)."""
    vol = hx * hy * hz
    # d/dx [-(1 - xi)/(hy hz)] = 1/(hx hy hz); d/dx [xi/(hy hz)] = 1/(hx hy hz); same for y, z
    return np.repeat((1.0 / vol)[:, None], 6, axis=1)


def volume_rule():
    x, y, z = np.meshgrid(GAUSS_X, GAUSS_X, GAUSS_X, indexing="ij")
    w = GAUSS_W[:, None, None] * GAUSS_W[None, :, None] * GAUSS_W[None, None, :]
    return x.ravel(), y.ravel(), z.ravel(), w.ravel()


def face_rule(f):
    """Reference points and weights (summing to 1) of the 3x3 rule on local face f."""
    s, t = np.meshgrid(GAUSS_X, GAUSS_X, indexing="ij")
    s, t = s.ravel(), t.ravel()
    w = (GAUSS_W[:, None] * GAUSS_W[None, :]).ravel()
    c = np.zeros_like(s) if f % 2 == 0 else np.ones_like(s)
    if f < 2:
        return c, s, t, w
    if f < 4:
        return s, c, t, w
    return s, t, c, w


def cell_data(mesh: BoxMesh, prob, cells=None):
    """Per-cell geometry and reference-state values in the oracle's cell order (or for ``cells``)."""
    sel = slice(None) if cells is None else np.asarray(cells)
    k = mesh.cell_layer[sel]
    col = (mesh.cell_iy * mesh.nx + mesh.cell_ix)[sel]
    hz = mesh.dz[k]
    hx = np.full(k.shape[0], mesh.dx)
    hy = np.full(k.shape[0], mesh.dy)
    return dict(
        hx=hx,
        hy=hy,
        hz=hz,
        thB=prob.theta_w[k, col],
        thT=prob.theta_w[k + 1, col],
        piB=prob.exner_hat_w[k, col],
        piT=prob.exner_hat_w[k + 1, col],
        pic=prob.exner_c[k, col],
        rhoc=prob.rho_c[k, col],
    )


def local_matrices(mesh: BoxMesh, prob, chunk: int = 8192, cells=None):
    """Cell matrices of the hybridised system for every cell (or only for ``cells``).

    Returns a dict of arrays (leading axis = cell):
      A  (7,7): [[M2 - Q22, G^b], [Q32 + M3rho M3^-1 D, M3Pi]] (velocity dofs 0..5, pressure 6)
      K  (6,6): k(v_a, nu_f)   - velocity rows, trace columns
      C  (6,6): c(v_a, nu_f)   - velocity rows, trace columns
      thF (6,): theta averaged over each face (used for the mixed facet term)
    and the separate blocks m2, q22, gb, d (the combined pressure row), q32,
    m3, m3rho, m3pi.
    """
    cd = cell_data(mesh, prob, cells)
    dt, tu, tr, tt = prob.dt, prob.tau_u, prob.tau_rho, prob.tau_theta
    cp, kappa = prob.cp, prob.kappa
    n = cd["hz"].shape[0]
    out = {key: np.zeros((n,) + shp) for key, shp in (
        ("A", (7, 7)), ("K", (6, 6)), ("C", (6, 6)), ("m2", (6, 6)), ("q22", (6, 6)),
        ("gb", (6,)), ("d", (6,)), ("q32", (6,)), ("m3", ()), ("m3rho", ()), ("m3pi", ()), ("thF", (6,)),
    )}
    qx, qy, qz, qw = volume_rule()
    for s0 in range(0, n, chunk):
        sl = slice(s0, min(n, s0 + chunk))
        hx, hy, hz = cd["hx"][sl], cd["hy"][sl], cd["hz"][sl]
        vol = hx * hy * hz
        thB, thT, piB, piT = cd["thB"][sl], cd["thT"][sl], cd["piB"][sl], cd["piT"][sl]
        pic, rhoc = cd["pic"][sl], cd["rhoc"][sl]
        v = rt0_values(qx, qy, qz, hx, hy, hz)  # (nc, nq, 6, 3)
        div = rt0_div(hx, hy, hz)  # (nc, 6)
        wq = qw[None, :] * vol[:, None]  # (nc, nq)
        theta_q = thB[:, None] * (1.0 - qz)[None, :] + thT[:, None] * qz[None, :]
        dth = (thT - thB) / hz
        dpi = (piT - piB) / hz
        # m2(w, u) = <w . u>   (mu = 0, Omega = 0)
        m2 = np.einsum("cq,cqad,cqbd->cab", wq, v, v)
        # q22(w, u) = tau_u tau_theta dt^2 < cp (z.w) dz Pihat (z.u) dz theta >
        q22 = tu * tt * dt * dt * cp * np.einsum(
            "cq,cqa,cqb->cab", wq * (dpi * dth)[:, None], v[:, :, :, 2], v[:, :, :, 2]
        )
        # g^b(w, Pi) = -tau_u dt cp < div(theta w) Pi >, Pi = 1 in the cell;
        # div(theta w) = theta div w + w_z d theta/dz  (theta varies only in z)
        divthw = theta_q[:, :, None] * div[:, None, :] + v[:, :, :, 2] * dth[:, None, None]
        gb = -tu * dt * cp * np.einsum("cq,cqa->ca", wq, divthw)
        # d(phi, u) = tau_rho dt < phi div(rho* u) >, rho* constant in the cell
        dD = tr * dt * rhoc[:, None] * np.einsum("cq,ca->ca", wq, div)
        # m3(phi, rho) = < phi rho >
        m3 = wq.sum(axis=1)
        # one-point (cell centre) rules for q32, m3^rho, m3^Pi
        vc = rt0_values(np.array([0.5]), np.array([0.5]), np.array([0.5]), hx, hy, hz)[:, 0]  # (nc, 6, 3)
        thc = 0.5 * (thB + thT)
        q32 = tt * dt * ((dth / thc)[:, None] * vc[:, :, 2]) * vol[:, None]
        m3rho = vol / rhoc
        m3pi = (1.0 - kappa) / kappa * vol / pic
        # facet forms: k(w, nu) = tau_u dt cp <[[theta w]] nu>, c(w, nu) = <[[w]] nu>
        Kmat = np.zeros((hx.shape[0], 6, 6))
        Cmat = np.zeros((hx.shape[0], 6, 6))
        thF = np.zeros((hx.shape[0], 6))
        area = np.stack([hy * hz, hy * hz, hx * hz, hx * hz, hx * hy, hx * hy], axis=1)
        for f in range(6):
            fx, fy, fz, fw = face_rule(f)
            vf = rt0_values(fx, fy, fz, hx, hy, hz)  # (nc, nqf, 6, 3)
            vn = np.einsum("cqad,d->cqa", vf, FACE_NORMALS[f])
            th_f = thB[:, None] * (1.0 - fz)[None, :] + thT[:, None] * fz[None, :]
            wf = fw[None, :] * area[:, f][:, None]
            Kmat[:, :, f] = tu * dt * cp * np.einsum("cq,cq,cqa->ca", wf, th_f, vn)
            Cmat[:, :, f] = np.einsum("cq,cqa->ca", wf, vn)
            thF[:, f] = np.einsum("cq,cq->c", wf, th_f) / area[:, f]
        drow = q32 + (m3rho / m3)[:, None] * dD
        A = np.zeros((hx.shape[0], 7, 7))
        A[:, :6, :6] = m2 - q22
        A[:, :6, 6] = gb
        A[:, 6, :6] = drow
        A[:, 6, 6] = m3pi
        for key, val in (("A", A), ("K", Kmat), ("C", Cmat), ("m2", m2), ("q22", q22), ("gb", gb),
                         ("d", drow), ("q32", q32), ("m3", m3), ("m3rho", m3rho), ("m3pi", m3pi),
                         ("thF", thF)):
            out[key][sl] = val
    return out
