"""Pins of the oracle on the extruded cubed sphere: mesh tables, the shell cell map, the cell
matrices on curved cells (with rotation), condensation, the mixed solve, conservation and the
two-level preconditioner (CPU only)."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.local import (local_matrices, local_matrices_mapped, shell_cells, shell_local_matrices, shell_map,
                          trilinear_map, cell_data)
from oracle.mesh import BoxMesh, TableMesh
from oracle.precond import lumped_velocity_mass
from oracle.problem import OracleProblem, cells_from_soa
from synth import make_box, make_sphere, make_rhs_sphere
from synth.sphere import cubed_sphere_tables


def spherical_triangle(a, b, c):
    """Solid angle of the spherical triangle with unit vertices a, b, c (Van Oosterom and
    Strackee, 1983)."""
    num = np.abs(np.einsum("cd,cd->c", a, np.cross(b, c)))
    den = 1 + np.einsum("cd,cd->c", a, b) + np.einsum("cd,cd->c", b, c) + np.einsum("cd,cd->c", c, a)
    return 2 * np.arctan2(num, den)


def consts_of(p):
    return dict(dt=p.dt, tau_u=p.tau_u, tau_rho=p.tau_rho, tau_theta=p.tau_theta, cp=p.cp, kappa=p.kappa)


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_cubed_sphere_tables(n):
    ce, ec, el, U = cubed_sphere_tables(n)
    ncol = 6 * n * n
    for s in range(2):
        assert np.array_equal(ce[el[s], ec[s]], np.arange(2 * ncol))
    assert np.all(ec[0] != ec[1])
    # Euler characteristic of the sphere: V - E + F = 2
    pts = np.round(np.concatenate([U[q].T for q in range(4)]), 12)
    V = np.unique(pts, axis=0).shape[0]
    assert V - 2 * ncol + ncol == 2
    # the two columns of an edge share its two corner points
    ends = {0: (0, 2), 1: (1, 3), 2: (0, 1), 3: (2, 3)}
    a = np.array([ends[f] for f in el[0]])
    b = np.array([ends[f] for f in el[1]])
    P = [U[a[:, i], :, ec[0]] for i in range(2)]
    Q = [U[b[:, i], :, ec[1]] for i in range(2)]
    same = np.minimum(np.abs(P[0] - Q[0]).max(1) + np.abs(P[1] - Q[1]).max(1),
                      np.abs(P[0] - Q[1]).max(1) + np.abs(P[1] - Q[0]).max(1))
    assert same.max() == 0.0
    # every column frame turns the same way seen from outside
    nrm = np.cross((U[1] - U[0]).T, (U[2] - U[0]).T)
    assert np.all(np.einsum("cd,cd->c", nrm, U.mean(axis=0).T) > 0)


def test_cubed_sphere_hierarchy():
    p = make_sphere(8, 2, mg_levels=3)
    for lf, lc in zip(p.levels[:-1], p.levels[1:]):
        par = lc.parent
        assert np.array_equal(np.bincount(par), np.full(lc.ncol, 4))
        # fine columns joined by an edge have the same coarse column or coarse columns that share
        # an edge; the local face of a fine edge on the boundary of its parent is the parent's
        ec, el = lf.edge_col, lf.edge_lf
        P0, P1 = par[ec[0]], par[ec[1]]
        cross = P0 != P1
        cf = lc.col_edge[el[0, cross], P0[cross]]
        assert np.array_equal(lc.edge_col[0, cf] + lc.edge_col[1, cf], P0[cross] + P1[cross])


def test_shell_map_derivatives_and_orthogonality():
    p = make_sphere(3, 2, mg_levels=1)
    m = TableMesh(p.nlev, p.col_edge, p.edge_col, p.edge_lf)
    U, r0, r1 = shell_cells(m, p)
    cmap = shell_map(U, r0, r1)
    rng = np.random.default_rng(1)
    q = rng.uniform(0.1, 0.9, (5, 3))
    x, J = cmap(q[:, 0], q[:, 1], q[:, 2])
    h = 1e-6
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        xp, _ = cmap(*(q + e).T)
        xm, _ = cmap(*(q - e).T)
        fd = (xp - xm) / (2 * h)
        assert np.abs(fd - J[..., d]).max() <= 1e-6 * np.abs(J[..., d]).max()
    r = r0[:, None] + q[None, :, 2] * (r1 - r0)[:, None]
    assert np.allclose(np.linalg.norm(x, axis=-1), r, rtol=1e-14)
    for d in range(2):
        cosang = np.einsum("cqd,cqd->cq", J[..., d], J[..., 2]) / (
            np.linalg.norm(J[..., d], axis=-1) * np.linalg.norm(J[..., 2], axis=-1))
        assert np.abs(cosang).max() <= 1e-13


def test_shell_cell_volumes():
    # exact volume of a cell: its solid angle (two spherical triangles: the edges are great-circle
    # arcs) times (r1^3 - r0^3) / 3; the 3-point Gauss rule converges at sixth order
    errs = []
    for n in (4, 8):
        p = make_sphere(n, 2, mg_levels=1)
        m = TableMesh(p.nlev, p.col_edge, p.edge_col, p.edge_lf)
        loc = shell_local_matrices(m, p)
        U, r0, r1 = shell_cells(m, p)
        om = spherical_triangle(U[:, 0], U[:, 1], U[:, 3]) + spherical_triangle(U[:, 0], U[:, 3], U[:, 2])
        assert abs(om.sum() / p.nlev - 4 * np.pi) <= 1e-12
        errs.append(np.abs(loc["vol"] / (om * (r1**3 - r0**3) / 3) - 1).max())
    assert errs[1] <= 2e-7
    assert errs[0] / errs[1] >= 30.0


def test_mapped_matrices_on_box_cells():
    # the cell-map code on axis-aligned cells (trilinear map, vertical +z) equals the box closed forms
    prob = make_box(nx=4, ny=3, nlev=3, dx=10e3, dy=7e3, dz=500.0, mg_levels=1, perturb=0.05)
    mesh = BoxMesh(prob.nx, prob.ny, prob.nlev, prob.dx, prob.dy, prob.z)
    ref = local_matrices(mesh, prob)
    X = np.zeros((mesh.ncell, 8, 3))
    for q in range(8):
        I, J, K = q & 1, (q >> 1) & 1, q >> 2
        X[:, q, 0] = (mesh.cell_ix + I) * prob.dx
        X[:, q, 1] = (mesh.cell_iy + J) * prob.dy
        X[:, q, 2] = prob.z[mesh.cell_layer + K]
    out = local_matrices_mapped(trilinear_map(X), cell_data(mesh, prob), consts_of(prob), radial=False)
    for key in ("A", "K", "C", "thF"):
        assert np.abs(out[key] - ref[key]).max() <= 1e-12 * np.abs(ref[key]).max(), key
    assert np.abs(out["cor"]).max() == 0.0


def _fields(nc, rng):
    thB = 300.0 + rng.uniform(0, 5, nc)
    return dict(thB=thB, thT=thB + rng.uniform(1, 5, nc), piB=0.9 + rng.uniform(0, 0.05, nc),
                piT=0.85 + rng.uniform(0, 0.04, nc), pic=rng.uniform(0.8, 1.0, nc), rhoc=rng.uniform(0.5, 1.2, nc))


def test_constant_fields_on_parallelepipeds():
    # an affine cell reproduces constant velocity fields: with dofs u_a = flux of U through face a,
    # the mass form gives |U|^2 |K|, the Coriolis form tau_u dt W . (2 Omega x U) |K| and q22
    # tau_u tau_theta dt^2 cp (z.W)(z.U) dz Pihat dz theta |K| (z fixed, fields linear in the cell)
    rng = np.random.default_rng(4)
    nc = 6
    A0 = rng.normal(size=(nc, 3, 3)) * 0.3 + np.diag([1e3, 2e3, 3e2])
    o = rng.normal(size=(nc, 3)) * 1e3
    X = np.empty((nc, 8, 3))
    for q in range(8):
        b = np.array([q & 1, (q >> 1) & 1, q >> 2], np.float64)
        X[:, q] = o + np.einsum("cde,e->cd", A0, b)
    Om = np.array([1e-4, -2e-4, 7e-5])
    fl = _fields(nc, rng)
    cs = dict(dt=900.0, tau_u=0.5, tau_rho=0.5, tau_theta=0.5, cp=1005.0, kappa=287.05 / 1005.0)
    out = local_matrices_mapped(trilinear_map(X), fl, cs, omega_vec=Om, radial=False)
    vol = np.abs(np.linalg.det(A0))
    assert np.allclose(out["vol"], vol, rtol=1e-13)
    # outward area vectors of the faces of the parallelepiped
    cols = [A0[:, :, 0], A0[:, :, 1], A0[:, :, 2]]
    area = [np.cross(cols[1], cols[2]), np.cross(cols[2], cols[0]), np.cross(cols[0], cols[1])]
    N = np.stack([-area[0], area[0], -area[1], area[1], -area[2], area[2]], axis=1)  # (nc, 6, 3)
    Uv, Wv = rng.normal(size=3), rng.normal(size=3)
    u = np.einsum("cfd,d->cf", N, Uv)
    w = np.einsum("cfd,d->cf", N, Wv)
    assert np.allclose(np.einsum("ca,cab,cb->c", u, out["m2"], u), vol * (Uv @ Uv), rtol=1e-12)
    cor = np.einsum("ca,cab,cb->c", w, out["cor"], u)
    assert np.allclose(cor, cs["tau_u"] * cs["dt"] * vol * (Wv @ np.cross(2 * Om, Uv)), rtol=1e-11)
    gz = np.linalg.inv(A0)[:, 2, :]  # grad of the vertical reference coordinate
    dth = (fl["thT"] - fl["thB"]) * gz[:, 2]
    dpi = (fl["piT"] - fl["piB"]) * gz[:, 2]
    q22 = cs["tau_u"] * cs["tau_theta"] * cs["dt"] ** 2 * cs["cp"] * Wv[2] * Uv[2] * dth * dpi * vol
    assert np.allclose(np.einsum("ca,cab,cb->c", w, out["q22"], u), q22, rtol=1e-11)


def test_curved_cell_identities_and_rotation_invariance():
    p = make_sphere(3, 3, mg_levels=1)
    m = TableMesh(p.nlev, p.col_edge, p.edge_col, p.edge_lf)
    loc = shell_local_matrices(m, p)
    cf = p.tau_u * p.dt * p.cp
    # unit flux per face; g^b = -diag(K) (divergence theorem); K = tau_u dt cp times the face mean
    assert np.abs(loc["C"] - np.eye(6)).max() <= 1e-13
    Kd = np.einsum("cii->ci", loc["K"])
    assert np.abs(loc["gb"] + Kd).max() <= 1e-14 * np.abs(Kd).max()
    assert np.abs(loc["K"] - Kd[:, :, None] * np.eye(6)).max() <= 1e-12 * np.abs(Kd).max()
    th = p.theta_w
    k, col = m.cell_layer, m.cell_col
    mean_side = 0.5 * (th[k, col] + th[k + 1, col])
    assert np.allclose(Kd[:, 0], cf * mean_side, rtol=1e-13)
    assert np.allclose(Kd[:, 4], cf * th[k, col], rtol=1e-13) and np.allclose(Kd[:, 5], cf * th[k + 1, col], rtol=1e-13)
    # the Coriolis block is skew; the mass block symmetric positive definite
    assert np.abs(loc["cor"] + loc["cor"].transpose(0, 2, 1)).max() <= 1e-14 * np.abs(loc["m2"]).max()
    np.linalg.cholesky(loc["m2"])
    # rotating the cell (and the vertical with it) changes nothing when Omega = 0
    U, r0, r1 = shell_cells(m, p)
    Q, _ = np.linalg.qr(np.random.default_rng(3).normal(size=(3, 3)))
    Q *= np.sign(np.linalg.det(Q))
    from oracle.local import shell_fields
    f = shell_fields(m, p)
    a = local_matrices_mapped(shell_map(U, r0, r1), f, consts_of(p))
    b = local_matrices_mapped(shell_map(U @ Q.T, r0, r1), f, consts_of(p))
    for key in ("A", "K", "C"):
        assert np.abs(a[key] - b[key]).max() <= 1e-11 * np.abs(a[key]).max(), key


@pytest.mark.parametrize("n,nlev", [(2, 2), (3, 2)])
def test_sphere_condensed_equals_dense_kkt(n, nlev):
    prob = make_sphere(n, nlev, mg_levels=1, perturb=0.05)
    o = OracleProblem(prob, with_precond=False)
    ruc, rpc = cells_from_soa(*make_rhs_sphere(prob, 3))
    lam, ub, pi, _ = o.hyb.solve_direct(ruc, rpc)
    lk, uk, pk = o.hyb.solve_kkt_dense(ruc, rpc)
    assert np.linalg.norm(lam - lk) <= 1e-10 * np.linalg.norm(lk)
    assert np.linalg.norm(ub - uk) <= 1e-10 * np.linalg.norm(uk)
    assert np.linalg.norm(pi - pk) <= 1e-10 * np.linalg.norm(pk)


@pytest.mark.parametrize("n,nlev", [(4, 3), (3, 4)])
def test_sphere_hybrid_equals_mixed_and_conserves(n, nlev):
    prob = make_sphere(n, nlev, mg_levels=1, perturb=0.05)
    o = OracleProblem(prob, with_precond=False)
    ruc, rpc = cells_from_soa(*make_rhs_sphere(prob, 11))
    u, pi = o.mixed.solve(ruc, rpc)
    lam, ub, pih, _ = o.hyb.solve_direct(ruc, rpc)
    ubm = o.mixed.broken_from_continuous(u)
    assert np.linalg.norm(pih - pi) <= 1e-10 * np.linalg.norm(pi)
    assert np.linalg.norm(ub - ubm) <= 1e-10 * np.linalg.norm(ubm)
    mesh = o.mesh
    flux = np.zeros(mesh.ntrace)
    np.add.at(flux, mesh.cell_faces.ravel(), ub.ravel())
    scale = np.abs(ub).max()
    assert np.abs(flux).max() <= 1e-11 * scale
    assert np.abs(ub[:, 4][mesh.cell_layer == 0]).max() <= 1e-11 * scale
    assert np.abs(ub[:, 5][mesh.cell_layer == prob.nlev - 1]).max() <= 1e-11 * scale
    assert abs(ub.sum()) <= 1e-11 * scale * mesh.ncell


def test_sphere_symmetric_case_and_rotation():
    # no stratification and no rotation: S symmetric positive definite; rotation adds a
    # nonsymmetric part that is odd in Omega, linear for small rates (tau_u dt 2 Omega << 1)
    base = dict(n=3, nlev=3, mg_levels=1, nbv=0.0)
    S = {}
    for om in (0.0, 1e-6, 2e-6):
        o = OracleProblem(make_sphere(omega_rot=om, **base), with_precond=False)
        S[om] = o.hyb.S.toarray()
    s0 = S[0.0]
    assert np.abs(s0 - s0.T).max() <= 1e-13 * np.abs(s0).max()
    np.linalg.cholesky(s0)
    k1 = S[1e-6] - S[1e-6].T
    k2 = S[2e-6] - S[2e-6].T
    assert np.abs(k1).max() > 1e-7 * np.abs(s0).max()
    assert np.abs(k2 - 2 * k1).max() <= 1e-3 * np.abs(k1).max()


def test_sphere_preconditioner_pieces():
    prob = make_sphere(8, 4, mg_levels=3)
    o = OracleProblem(prob)
    ml = lumped_velocity_mass(o.mixed)
    assert ml.min() > 0
    H = o.H
    off = H - sp.diags(H.diagonal())
    assert off.max() <= 0.0
    assert np.allclose(np.asarray(H.sum(axis=1)).ravel(), o.loc["m3pi"], rtol=1e-9)
    for h in o.pc.mg.H:
        assert np.diff(h.indptr).max() <= 7
        assert np.asarray(h.sum(axis=1)).ravel().min() > 0
    # eigenvalues of H_z^-1 H on the coarsest level inside the Chebyshev interval's upper end
    Hc = o.pc.mg.H[-1].toarray()
    Hz = o.pc.mg.Hz[-1].toarray()
    ev = np.linalg.eigvals(np.linalg.solve(Hz, Hc)).real
    assert ev.min() > 0 and ev.max() < 2.0


def test_sphere_two_level_fgmres():
    prob = make_sphere(8, 6, mg_levels=3)
    o = OracleProblem(prob)
    ruc, rpc = cells_from_soa(*make_rhs_sphere(prob, 0))
    lam, _, _, B = o.hyb.solve_direct(ruc, rpc)
    x, hist, its, conv = o.solve_fgmres(B, rtol=1e-10)
    assert conv and its <= 15
    assert np.linalg.norm(x - lam) <= 1e-8 * np.linalg.norm(lam)
    _, _, its0, _ = o.solve_fgmres(B, rtol=1e-8, maxit=100, precondition=False)
    assert its0 >= 100
