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


# ---------------------------------------------------------------------------------------------
# Curved cells (the extruded cubed sphere): the same forms under a general cell map
# ---------------------------------------------------------------------------------------------


def trilinear(xi, eta, zeta):
    """Trilinear shape functions of the 8 corners q = I + 2 J + 4 K at reference points and their
    reference gradients: arrays (nq, 8) and (nq, 8, 3)."""
    p = np.stack([xi, eta, zeta], axis=1)  # (nq, 3)
    N = np.ones((p.shape[0], 8))
    dN = np.ones((p.shape[0], 8, 3))
    for q in range(8):
        bits = (q & 1, (q >> 1) & 1, (q >> 2) & 1)
        for d in range(3):
            f = p[:, d] if bits[d] else 1.0 - p[:, d]
            df = 1.0 if bits[d] else -1.0
            N[:, q] *= f
            for e in range(3):
                dN[:, q, e] *= df if e == d else f
    return N, dN


def trilinear_map(X):
    """The trilinear cell map through corners X (nc, 8, 3): returns map(xi, eta, zeta) -> (x, J)
    with x (nc, nq, 3) and J[..., d, e] = d x_d / d xi_e."""
    X = np.asarray(X, np.float64)

    def m(xi, eta, zeta):
        N, dN = trilinear(xi, eta, zeta)
        return np.einsum("qa,cad->cqd", N, X), np.einsum("qae,cad->cqde", dN, X)

    return m


def shell_map(U, r0, r1):
    """The cell map of an extruded cubed-sphere cell: x = r(zeta) u(xi, eta) with
    r = r0 + zeta (r1 - r0) and u = p / |p|, p the bilinear interpolation of the column's corner
    unit vectors U (nc, 4, 3) (corner I + 2 J at (xi, eta) = (I, J)).  Bottom and top faces lie on
    spheres, the side faces in planes through the centre (great-circle edges), and the vertical
    direction d x / d zeta is radial, orthogonal to the two horizontal ones."""
    U = np.asarray(U, np.float64)
    r0, r1 = np.asarray(r0, np.float64), np.asarray(r1, np.float64)

    def m(xi, eta, zeta):
        w = np.stack([(1 - xi) * (1 - eta), xi * (1 - eta), (1 - xi) * eta, xi * eta], axis=1)  # (nq, 4)
        dwx = np.stack([-(1 - eta), 1 - eta, -eta, eta], axis=1)
        dwy = np.stack([-(1 - xi), -xi, 1 - xi, xi], axis=1)
        p = np.einsum("qa,cad->cqd", w, U)
        px = np.einsum("qa,cad->cqd", dwx, U)
        py = np.einsum("qa,cad->cqd", dwy, U)
        npn = np.linalg.norm(p, axis=-1, keepdims=True)
        u = p / npn
        ux = (px - u * np.einsum("cqd,cqd->cq", u, px)[..., None]) / npn
        uy = (py - u * np.einsum("cqd,cqd->cq", u, py)[..., None]) / npn
        r = r0[:, None] + zeta[None, :] * (r1 - r0)[:, None]
        x = r[..., None] * u
        J = np.stack([r[..., None] * ux, r[..., None] * uy, (r1 - r0)[:, None, None] * u], axis=-1)
        return x, J

    return m


def local_matrices_mapped(cmap, fields, consts, omega_vec=None, radial=True):
    """Cell matrices of the hybridised system on cells given by a cell map ``cmap`` of the unit
    cube (``trilinear_map`` or ``shell_map``).

    The lowest-order broken Raviart-Thomas functions are the reference ones (unit outward flux
    through their own face of the unit cube) mapped by the contravariant Piola transform
    v = J v_hat / det J, so every velocity dof is still the flux through its face.  W_theta fields
    are linear in the vertical reference coordinate; W3 functions are constant.  The vertical unit
    vector z_hat is the radial direction x / |x| (``radial``) or +z.  Forms of Sec. 2.2: the
    velocity mass with the Coriolis term tau_u dt <w . 2 Omega x u> (``omega_vec``, the rotation
    vector; the mu term is read as zero), q22 with z_hat and d/dz = z_hat . grad, g^b, d, m3 by
    the 3-point Gauss rule in each direction (weights det J); q32, m3^rho and m3^Pi by the
    one-point rule at the reference centre (weight det J there); k and c over the faces with the
    3x3 rule and the physical surface element (cross product of the face's tangent vectors).

    fields: dict of (nc,) arrays thB, thT, piB, piT (theta* and the projected Exner pressure at
    the bottom / top faces), pic, rhoc; consts: dict dt, tau_u, tau_rho, tau_theta, cp, kappa.
    Returns the same dict as ``local_matrices`` plus ``cor`` (the Coriolis block, included in A)
    and ``vol``.
    """
    dt, tu, tr, tt = consts["dt"], consts["tau_u"], consts["tau_rho"], consts["tau_theta"]
    cp, kappa = consts["cp"], consts["kappa"]
    thB, thT, piB, piT = fields["thB"], fields["thT"], fields["piB"], fields["piT"]
    pic, rhoc = fields["pic"], fields["rhoc"]
    nc = thB.shape[0]
    Om = np.zeros(3) if omega_vec is None else np.asarray(omega_vec, np.float64)

    def geometry(xi, eta, zeta):
        x, J = cmap(xi, eta, zeta)
        det = np.linalg.det(J)
        Jinv = np.linalg.inv(J)
        vhat = rt0_values(xi, eta, zeta, np.ones(1), np.ones(1), np.ones(1))[0]  # (nq, 6, 3)
        v = np.einsum("cqde,qae->cqad", J, vhat) / det[:, :, None, None]
        if radial:
            zh = x / np.linalg.norm(x, axis=-1, keepdims=True)
        else:
            zh = np.broadcast_to(np.array([0.0, 0.0, 1.0]), x.shape)
        gzeta = Jinv[:, :, 2, :]  # grad of the vertical reference coordinate
        return J, det, v, zh, gzeta

    qx, qy, qz, qw = volume_rule()
    J, det, v, zh, gz = geometry(qx, qy, qz)
    wq = qw[None, :] * det  # (nc, nq)
    div = 1.0 / det  # (nc, nq), the same for all six functions
    th_q = thB[:, None] * (1.0 - qz)[None, :] + thT[:, None] * qz[None, :]
    grad_th = (thT - thB)[:, None, None] * gz  # (nc, nq, 3)
    dzth = np.einsum("cqd,cqd->cq", zh, grad_th)
    dzpi = np.einsum("cqd,cqd->cq", zh, (piT - piB)[:, None, None] * gz)
    vz = np.einsum("cqad,cqd->cqa", v, zh)
    m2 = np.einsum("cq,cqad,cqbd->cab", wq, v, v)
    cv = 2.0 * np.cross(np.broadcast_to(Om, v.shape), v)  # 2 Omega x v_b
    cor = tu * dt * np.einsum("cq,cqad,cqbd->cab", wq, v, cv)
    q22 = tu * tt * dt * dt * cp * np.einsum("cq,cqa,cqb->cab", wq * dzpi * dzth, vz, vz)
    divthw = th_q[:, :, None] * div[:, :, None] + np.einsum("cqad,cqd->cqa", v, grad_th)
    gb = -tu * dt * cp * np.einsum("cq,cqa->ca", wq, divthw)
    dD = tr * dt * rhoc[:, None] * np.einsum("cq,cq->c", wq, div)[:, None] * np.ones((1, 6))
    m3 = wq.sum(axis=1)
    # one-point rule at the reference centre
    h = np.array([0.5])
    _, detc, vc, zc, gzc = geometry(h, h, h)
    detc, vc, zc, gzc = detc[:, 0], vc[:, 0], zc[:, 0], gzc[:, 0]
    thc = 0.5 * (thB + thT)
    dzth_c = (thT - thB) * np.einsum("cd,cd->c", zc, gzc)
    q32 = tt * dt * (dzth_c / thc)[:, None] * np.einsum("cad,cd->ca", vc, zc) * detc[:, None]
    m3rho = detc / rhoc
    m3pi = (1.0 - kappa) / kappa * detc / pic
    Kmat = np.zeros((nc, 6, 6))
    Cmat = np.zeros((nc, 6, 6))
    thF = np.zeros((nc, 6))
    tang = {0: (1, 2), 1: (1, 2), 2: (2, 0), 3: (2, 0), 4: (0, 1), 5: (0, 1)}
    for f in range(6):
        fx, fy, fz, fw = face_rule(f)
        Jf, _, vf, _, _ = geometry(fx, fy, fz)
        t1, t2 = tang[f]
        nds = np.cross(Jf[:, :, :, t1], Jf[:, :, :, t2]) * (1.0 if f % 2 else -1.0)  # outward
        flux = np.einsum("cqad,cqd->cqa", vf, nds) * fw[None, :, None]
        th_f = thB[:, None] * (1.0 - fz)[None, :] + thT[:, None] * fz[None, :]
        Kmat[:, :, f] = tu * dt * cp * np.einsum("cq,cqa->ca", th_f, flux)
        Cmat[:, :, f] = flux.sum(axis=1)
        thF[:, f] = Kmat[:, f, f] / (tu * dt * cp)
    drow = q32 + (m3rho / m3)[:, None] * dD
    A = np.zeros((nc, 7, 7))
    A[:, :6, :6] = m2 + cor - q22
    A[:, :6, 6] = gb
    A[:, 6, :6] = drow
    A[:, 6, 6] = m3pi
    return dict(A=A, K=Kmat, C=Cmat, m2=m2, q22=q22, cor=cor, gb=gb, d=drow, q32=q32, m3=m3,
                m3rho=m3rho, m3pi=m3pi, thF=thF, vol=m3)


def shell_cells(mesh, prob, cells=None):
    """Corner unit vectors (nc, 4, 3), bottom and top radii (nc,) of cells of a cubed sphere."""
    sel = slice(None) if cells is None else np.asarray(cells)
    k = mesh.cell_layer[sel]
    col = mesh.cell_col[sel]
    U = np.stack([prob.corners[q][:, col].T for q in range(4)], axis=1)
    return U, prob.radius[k], prob.radius[k + 1]


def shell_fields(mesh, prob, cells=None):
    sel = slice(None) if cells is None else np.asarray(cells)
    k = mesh.cell_layer[sel]
    col = mesh.cell_col[sel]
    return dict(thB=prob.theta_w[k, col], thT=prob.theta_w[k + 1, col], piB=prob.exner_hat_w[k, col],
                piT=prob.exner_hat_w[k + 1, col], pic=prob.exner_c[k, col], rhoc=prob.rho_c[k, col])


def shell_local_matrices(mesh, prob, cells=None, chunk=4096):
    """Cell matrices of every cell (or of ``cells``) of an extruded cubed sphere (``shell_map``),
    rotating about the polar (+z) axis at prob.omega_rot."""
    idx = np.arange(mesh.ncell) if cells is None else np.asarray(cells)
    consts = dict(dt=prob.dt, tau_u=prob.tau_u, tau_rho=prob.tau_rho, tau_theta=prob.tau_theta, cp=prob.cp,
                  kappa=prob.kappa)
    out = None
    for s0 in range(0, idx.shape[0], chunk):
        sel = idx[s0 : s0 + chunk]
        U, r0, r1 = shell_cells(mesh, prob, sel)
        part = local_matrices_mapped(shell_map(U, r0, r1), shell_fields(mesh, prob, sel), consts,
                                     omega_vec=np.array([0.0, 0.0, prob.omega_rot]))
        if out is None:
            out = {k: np.zeros((idx.shape[0],) + v.shape[1:]) for k, v in part.items()}
        for k, v in part.items():
            out[k][s0 : s0 + sel.shape[0]] = v
    return out
