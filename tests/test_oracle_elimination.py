"""Pins of the oracle's elimination of theta' and rho' and their back-substitution (CPU only).

The four-field system (u, rho, theta', Pi) assembled and solved by sparse LU must give the same
fields as the elimination (Sec. 2.1, 2.2), the 2x2 solve and the back-substitution; the right-hand
side change and the recovered theta' match closed forms worked out by hand on box and cubed-sphere
cells; invariants hold where the mathematics fixes them."""

import numpy as np
import pytest

from oracle.elimination import FourFieldSystem, back_substitute, box_map, eliminate_rhs
from oracle.local import local_matrices, shell_cells, shell_fields, shell_map
from oracle.mesh import BoxMesh, TableMesh
from synth import make_box, make_rhs, make_sphere, make_rhs_sphere


def _residuals(prob, seed):
    """A seeded four-field residual: r_u^b, r_rho, r_theta (facets), r_Pi in cell order."""
    rng = np.random.default_rng(seed)
    L, ncol = prob.nlev, prob.ncol
    r_ub = rng.standard_normal((L * ncol, 6))
    r_rho = rng.standard_normal(L * ncol) * 1e-2
    r_th = rng.standard_normal((L + 1, ncol))
    r_pi = rng.standard_normal(L * ncol) * 1e-3
    return r_ub, r_rho, r_th, r_pi


def _box(prob):
    mesh = BoxMesh(prob.nx, prob.ny, prob.nlev, prob.dx, prob.dy, prob.z)
    k = mesh.cell_layer
    col = mesh.cell_iy * mesh.nx + mesh.cell_ix
    fields = dict(thB=prob.theta_w[k, col], thT=prob.theta_w[k + 1, col], piB=prob.exner_hat_w[k, col],
                  piT=prob.exner_hat_w[k + 1, col], rhoc=prob.rho_c[k, col], pic=prob.exner_c[k, col])
    consts = dict(dt=prob.dt, tau_u=prob.tau_u, tau_rho=prob.tau_rho, tau_theta=prob.tau_theta, cp=prob.cp)
    cmap = box_map(np.full(mesh.ncell, mesh.dx), np.full(mesh.ncell, mesh.dy), mesh.dz[k])
    return mesh, k, col, fields, consts, cmap


@pytest.mark.parametrize(
    "kw",
    [
        dict(nx=3, ny=3, nlev=3, dx=10e3, dz=1000.0, mg_levels=1, perturb=0.05),
        dict(nx=4, ny=3, nlev=5, dx=8e3, dy=6e3, ztop=12e3, stretch="quadratic", mg_levels=1, perturb=0.1, seed=2),
    ],
)
def test_four_field_system_equals_elimination_solve_and_back_substitution(kw):
    from oracle.hybrid import HybridSystem
    from oracle.mixed import MixedSystem

    prob = make_box(**kw)
    mesh, k, col, fields, consts, cmap = _box(prob)
    loc = local_matrices(mesh, prob)
    four = FourFieldSystem(mesh, prob, loc)
    r_ub, r_rho, r_th, r_pi = _residuals(prob, 7)
    rthB, rthT = r_th[k, col], r_th[k + 1, col]
    u4, rho4, th4, pi4 = four.solve(r_ub, r_rho, rthB, rthT, r_pi)
    # elimination, the 2x2 solve (mixed system by LU, and the hybridised system), back-substitution
    r_ub_bar, r_pi_bar = eliminate_rhs(cmap, False, fields, consts, r_ub, r_rho, rthB, rthT, r_pi)
    mixed = MixedSystem(mesh, loc, prob)
    u2, pi2 = mixed.solve(r_ub_bar, r_pi_bar)
    ub2 = mixed.broken_from_continuous(u2)
    rho2, th2 = back_substitute(cmap, False, fields, consts, r_rho, rthB, rthT, ub2)
    _, ubh, pih, _ = HybridSystem(mesh, loc).solve_direct(r_ub_bar, r_pi_bar)
    rhoh, thh = back_substitute(cmap, False, fields, consts, r_rho, rthB, rthT, ubh)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)  # noqa: E731
    errs = [rel(u2, u4), rel(pi2, pi4), rel(rho2, rho4), rel(th2, th4), rel(ubh, ub2), rel(pih, pi4),
            rel(rhoh, rho4), rel(thh, th4)]
    assert max(errs) <= 1e-10, errs
    # every term matters: dropping the theta' coupling from the momentum row changes the answer
    r_plain, _ = eliminate_rhs(cmap, False, fields, dict(consts, tau_u=0.0), r_ub, r_rho, rthB, rthT, r_pi)
    u_bad, _ = mixed.solve(r_plain, r_pi_bar)
    assert rel(u_bad, u4) > 1e-3


def test_rhs_change_closed_form_box_and_sphere():
    """On a cell with unit-flux basis functions the momentum change is
    -/+ tau_u dt c_p (Pihat_T - Pihat_B) (r_B/3 + r_T/6 | r_B/6 + r_T/3) on the bottom / top facet
    and zero on the sides (the integral of (z.v_F) r_theta d/dz Pihat does not depend on the cell
    shape); the pressure dual gains w_c (r_theta(c) / theta*(c) + r_rho / rho*)."""
    cases = []
    prob = make_box(nx=3, ny=2, nlev=4, dx=7e3, dy=5e3, ztop=9e3, stretch="quadratic", mg_levels=1, perturb=0.1)
    mesh, k, col, fields, consts, cmap = _box(prob)
    cases.append((prob, k, col, fields, consts, cmap, False, mesh.dx * mesh.dy * mesh.dz[k]))
    sph = make_sphere(3, 3, mg_levels=1, perturb=0.05)
    tm = TableMesh(sph.nlev, sph.col_edge, sph.edge_col, sph.edge_lf)
    U, r0, r1 = shell_cells(tm, sph)
    f = shell_fields(tm, sph)
    consts_s = dict(dt=sph.dt, tau_u=sph.tau_u, tau_rho=sph.tau_rho, tau_theta=sph.tau_theta, cp=sph.cp)
    # det J at the reference centre by hand: (r1 - r0) r_c^2 [u_xi x u_eta] . u at (1/2, 1/2)
    p = U.mean(axis=1)
    npn = np.linalg.norm(p, axis=1, keepdims=True)
    u = p / npn
    px = 0.5 * (U[:, 1] - U[:, 0] + U[:, 3] - U[:, 2])
    py = 0.5 * (U[:, 2] - U[:, 0] + U[:, 3] - U[:, 1])
    ux = (px - u * np.einsum("cd,cd->c", u, px)[:, None]) / npn
    uy = (py - u * np.einsum("cd,cd->c", u, py)[:, None]) / npn
    tri = np.einsum("cd,cd->c", np.cross(ux, uy), u)
    wc = (r1 - r0) * (0.5 * (r0 + r1)) ** 2 * tri
    cases.append((sph, tm.cell_layer, tm.cell_col, f, consts_s, shell_map(U, r0, r1), True, wc))
    for prob_, k, col, fields, consts, cmap, radial, wc in cases:
        r_ub, r_rho, r_th, r_pi = _residuals(prob_, 3)
        rB, rT = r_th[k, col], r_th[k + 1, col]
        r_ub_bar, r_pi_bar = eliminate_rhs(cmap, radial, fields, consts, r_ub, r_rho, rB, rT, r_pi)
        eu = prob_.tau_u * prob_.dt * prob_.cp * (fields["piT"] - fields["piB"])
        dref = np.zeros_like(r_ub)
        dref[:, 4] = eu * (rB / 3 + rT / 6)
        dref[:, 5] = -eu * (rB / 6 + rT / 3)
        np.testing.assert_allclose(r_ub_bar - r_ub, dref, rtol=1e-11, atol=1e-13 * np.abs(dref).max())
        thc = 0.5 * (fields["thB"] + fields["thT"])
        pref = wc * (r_pi + 0.5 * (rB + rT) / thc + r_rho / fields["rhoc"])
        np.testing.assert_allclose(r_pi_bar, pref, rtol=1e-11)


def test_theta_recovery_closed_form_and_invariants():
    """theta'_T = r_T - tau_theta dt (theta_T - theta_B) / (r1 - r0) * u_T / A_T with A_T the area
    density at the top facet centre (hx hy on the box, r1^2 [u_xi x u_eta] . u on the sphere), and
    theta'_B likewise with -u_B / A_B; no residual of theta or rho leaves the right-hand sides
    unchanged; theta* constant gives theta' = r_theta; a uniform rho* conserves the mass of rho'."""
    prob = make_box(nx=3, ny=3, nlev=4, dx=6e3, dy=4e3, dz=500.0, mg_levels=1, perturb=0.05)
    mesh, k, col, fields, consts, cmap = _box(prob)
    rng = np.random.default_rng(5)
    ub = rng.standard_normal((mesh.ncell, 6))
    r_ub, r_rho, r_th, r_pi = _residuals(prob, 4)
    rB, rT = r_th[k, col], r_th[k + 1, col]
    rho, th = back_substitute(cmap, False, fields, consts, r_rho, rB, rT, ub)
    dth = prob.tau_theta * prob.dt * (fields["thT"] - fields["thB"]) / mesh.dz[k]
    area = mesh.dx * mesh.dy
    np.testing.assert_allclose(th[:, 1], rT - dth * ub[:, 5] / area, rtol=1e-12)
    np.testing.assert_allclose(th[:, 0], rB + dth * ub[:, 4] / area, rtol=1e-12)
    vol = mesh.dx * mesh.dy * mesh.dz[k]
    np.testing.assert_allclose(rho, r_rho - prob.tau_rho * prob.dt * fields["rhoc"] * ub.sum(axis=1) / vol,
                               rtol=1e-12)
    zero = np.zeros(mesh.ncell)
    rb0, rp0 = eliminate_rhs(cmap, False, fields, consts, r_ub, zero, zero, zero, r_pi)
    assert np.array_equal(rb0, r_ub)
    np.testing.assert_allclose(rp0, vol * r_pi, rtol=1e-13)
    # theta* constant (N = 0): no buoyancy, theta' = r_theta
    p0 = make_box(nx=3, ny=3, nlev=4, dx=6e3, dz=500.0, mg_levels=1, nbv=0.0)
    m0, k0, c0, f0, cs0, cm0 = _box(p0)
    _, th0 = back_substitute(cm0, False, f0, cs0, zero, rB, rT, ub)
    np.testing.assert_allclose(th0, np.stack([rB, rT], axis=1), rtol=0, atol=1e-15)
    # sphere: the area density at the facet centres by hand
    sph = make_sphere(2, 3, mg_levels=1)
    tm = TableMesh(sph.nlev, sph.col_edge, sph.edge_col, sph.edge_lf)
    U, r0, r1 = shell_cells(tm, sph)
    f = shell_fields(tm, sph)
    consts_s = dict(dt=sph.dt, tau_u=sph.tau_u, tau_rho=sph.tau_rho, tau_theta=sph.tau_theta, cp=sph.cp)
    ubs = rng.standard_normal((tm.ncell, 6))
    rts = rng.standard_normal((sph.nlev + 1, sph.ncol))
    rBs, rTs = rts[tm.cell_layer, tm.cell_col], rts[tm.cell_layer + 1, tm.cell_col]
    _, ths = back_substitute(shell_map(U, r0, r1), True, f, consts_s, np.zeros(tm.ncell), rBs, rTs, ubs)
    p = U.mean(axis=1)
    npn = np.linalg.norm(p, axis=1, keepdims=True)
    u = p / npn
    px = 0.5 * (U[:, 1] - U[:, 0] + U[:, 3] - U[:, 2])
    py = 0.5 * (U[:, 2] - U[:, 0] + U[:, 3] - U[:, 1])
    ux = (px - u * np.einsum("cd,cd->c", u, px)[:, None]) / npn
    uy = (py - u * np.einsum("cd,cd->c", u, py)[:, None]) / npn
    tri = np.einsum("cd,cd->c", np.cross(ux, uy), u)
    dths = sph.tau_theta * sph.dt * (f["thT"] - f["thB"]) / (r1 - r0)
    np.testing.assert_allclose(ths[:, 1], rTs - dths * ubs[:, 5] / (r1**2 * tri), rtol=1e-11)
    np.testing.assert_allclose(ths[:, 0], rBs + dths * ubs[:, 4] / (r0**2 * tri), rtol=1e-11)


def test_density_mass_conservation():
    """With rho* uniform, the recovered rho' has the mass of r_rho (fluxes of a continuous velocity
    with no flow through lid and ground cancel)."""
    from oracle.mixed import MixedSystem

    prob = make_box(nx=4, ny=4, nlev=3, dx=5e3, dz=400.0, mg_levels=1, rho_scale_height=1e300, perturb=0.05)
    mesh, k, col, fields, consts, cmap = _box(prob)
    loc = local_matrices(mesh, prob)
    r_ub, r_rho, r_th, r_pi = _residuals(prob, 9)
    rB, rT = r_th[k, col], r_th[k + 1, col]
    rb, rp = eliminate_rhs(cmap, False, fields, consts, r_ub, r_rho, rB, rT, r_pi)
    mixed = MixedSystem(mesh, loc, prob)
    u, _ = mixed.solve(rb, rp)
    rho, _ = back_substitute(cmap, False, fields, consts, r_rho, rB, rT, mixed.broken_from_continuous(u))
    vol = mesh.dx * mesh.dy * mesh.dz[k]
    assert abs((vol * rho).sum() - (vol * r_rho).sum()) <= 1e-12 * np.abs(vol * r_rho).sum()
    assert np.abs(rho - r_rho).max() > 1e-6 * np.abs(r_rho).max()  # the flux term is not zero
