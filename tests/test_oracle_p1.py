"""Pins of the p = 1 oracle (CPU only): bases, quadrature, the p = 0 forms embedded in p = 1, the
table of unknowns, the dense hybridised system, equivalence with the mixed system, continuity."""

import numpy as np
import pytest

from oracle import local as p0
from oracle import p1
from oracle.mesh import BoxMesh
from synth import make_box


def _mesh(nx=3, ny=2, nlev=3, **kw):
    prob = make_box(nx=nx, ny=ny, nlev=nlev, dx=kw.pop("dx", 5e3), dz=kw.pop("dz", 250.0), mg_levels=1, **kw)
    return prob, BoxMesh(prob.nx, prob.ny, prob.nlev, prob.dx, prob.dy, prob.z)


def _rhs(mesh, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((mesh.ncell, p1.NU)), rng.standard_normal((mesh.ncell, p1.NP))


def test_table_of_unknowns(golden_dir):
    """44 x 44 mixed and 24 x 24 hybridised local matrices; 12 trace dofs per cell away from the
    lid and ground (the paper's table of unknowns, p = 1 row)."""
    rows = [ln.split() for ln in open(f"{golden_dir}/table5_dofs.txt") if ln.strip() and not ln.startswith("#")]
    p1row = [r for r in rows if r[0] == "1"][0]
    prob, mesh = _mesh()
    loc = p1.local_matrices(mesh, prob)
    n_lambda, mixed_local, hybrid_local = int(p1row[4]), int(p1row[5]), int(p1row[6])
    assert loc["A"].shape[1:] == (mixed_local, mixed_local)
    assert p1.cell_trace_operator(loc).shape[1:] == (hybrid_local, hybrid_local)
    h = p1.HybridP1(mesh, loc)
    assert h.ntrace == 4 * (mesh.ncol * (mesh.nlev + 1) + 2 * mesh.ncol * mesh.nlev)
    assert (h.ntrace - 4 * mesh.ncol) / mesh.ncell == n_lambda


def test_basis_nodal_identities():
    """Face function (f, i) has outward normal component 1 at face point i of face f and 0 at every
    other face point; interior functions have no normal component on any face; the DG1 and trace
    functions are nodal at the Gauss points."""
    h = (np.array([3.0]), np.array([2.0]), np.array([0.5]))
    for f in range(6):
        pf, _ = p1.face_points(f, 2)
        v, _ = p1.rt1_values(pf, h)
        vn = p1.FACE_SIGN[f] * v[0, :, :, p1.FACE_DIR[f]]  # (4 points, 36)
        expect = np.zeros((4, p1.NU))
        expect[np.arange(4), 4 * f + np.arange(4)] = 1.0
        np.testing.assert_allclose(vn, expect, atol=1e-14)
    pn, _ = p1.volume_rule(2)
    np.testing.assert_allclose(p1.dg1_values(pn), np.eye(8), atol=1e-14)


def test_divergence_theorem_per_basis_function():
    """int_K div w = sum_f int_f w . n for every velocity function, from the assembled forms:
    d / (tau_rho dt rho*) summed over the DG1 partition of unity against C summed over the trace
    partition of unity."""
    prob, mesh = _mesh(dx=7e3, dz=300.0)
    loc = p1.local_matrices(mesh, prob)
    cd = p0.cell_data(mesh, prob)
    vol_div = loc["d"].sum(axis=1) / (prob.tau_rho * prob.dt * cd["rhoc"][:, None])
    flux = loc["C"].sum(axis=2)
    np.testing.assert_allclose(vol_div, flux, rtol=1e-12, atol=1e-12 * np.abs(flux).max())


def test_quadrature_rule_is_exact():
    """The n = p + 3 = 4 point rule integrates every form exactly: n = 6 gives the same matrices."""
    prob, mesh = _mesh(nx=2, ny=2, nlev=3, perturb=0.05)
    a, b = p1.local_matrices(mesh, prob, n_quad=4), p1.local_matrices(mesh, prob, n_quad=6)
    for key in ("m2", "q22", "gb", "d", "m3", "K", "C", "A"):
        np.testing.assert_allclose(a[key], b[key], rtol=1e-12, atol=1e-12 * np.abs(b[key]).max(), err_msg=key)


def _embedding(hx, hy, hz):
    """RT0 functions (unit outward flux) written in the RT1 dofs: the outward normal component at
    the face points and the component at the interior nodes, evaluated with the p = 0 module."""
    E = np.zeros((p1.NU, 6))
    for j, (d, a, (t1, t2), sgn) in enumerate(p1.RT1):
        pt = [0.0, 0.0, 0.0]
        pt[d] = p1.Q3[a]
        u, w = p1.TANG[d]
        pt[u], pt[w] = p1.G2[t1], p1.G2[t2]
        v = p0.rt0_values(np.array([pt[0]]), np.array([pt[1]]), np.array([pt[2]]), np.array([hx]), np.array([hy]),
                          np.array([hz]))[0, 0]  # (6, 3)
        E[j] = sgn * v[:, d]
    return E


def test_p0_fields_embedded_in_p1_reproduce_the_p0_forms():
    """RT0 c RT1, DG0 c DG1 and the constant trace c Q1 trace: every form of the p = 1 module applied
    to the embedded p = 0 functions equals the (separately pinned) p = 0 cell matrix.  q32 uses the
    nodal rule of W3, so at p = 1 it is the two-point Gauss rule in the vertical of the p = 0
    integrand instead of its centre value; it is checked against that."""
    prob, mesh = _mesh(nx=2, ny=2, nlev=3, perturb=0.05, dx=6e3, dz=400.0)
    l1, l0 = p1.local_matrices(mesh, prob), p0.local_matrices(mesh, prob)
    cd = p0.cell_data(mesh, prob)
    one8 = np.ones(8)
    T = np.zeros((p1.NF, 6))
    for f in range(6):
        T[4 * f: 4 * f + 4, f] = 1.0
    for c in range(mesh.ncell):
        E = _embedding(cd["hx"][c], cd["hy"][c], cd["hz"][c])
        chk = {
            "m2": (E.T @ l1["m2"][c] @ E, l0["m2"][c]),
            "q22": (E.T @ l1["q22"][c] @ E, l0["q22"][c]),
            "gb": (E.T @ l1["gb"][c] @ one8, l0["gb"][c]),
            # the p = 0 module's "d" is the combined pressure row q32 + M3rho M3^-1 D
            "drow - q32": (one8 @ (l1["A"][c][p1.NU:, : p1.NU] - l1["q32"][c]) @ E, l0["d"][c] - l0["q32"][c]),
            # every RT0 function has unit outward flux, so d(1, v) = tau_rho dt rho*
            "d": (one8 @ l1["d"][c] @ E, np.full(6, prob.tau_rho * prob.dt * cd["rhoc"][c])),
            "m3": (one8 @ l1["m3"][c] @ one8, l0["m3"][c]),
            "m3rho": (one8 @ l1["m3rho"][c] @ one8, l0["m3rho"][c]),
            "m3pi": (one8 @ l1["m3pi"][c] @ one8, l0["m3pi"][c]),
            "K": (E.T @ l1["K"][c] @ T, l0["K"][c]),
            "C": (E.T @ l1["C"][c] @ T, l0["C"][c]),
        }
        for key, (got, want) in chk.items():
            np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-12 * np.abs(want).max() + 1e-300,
                                       err_msg=f"{key} cell {c}")
        # q32 with the two-point Gauss rule in z of the p = 0 integrand tau_theta dt v_z dtheta/theta
        hx, hy, hz = cd["hx"][c], cd["hy"][c], cd["hz"][c]
        dth = (cd["thT"][c] - cd["thB"][c]) / hz
        want = np.zeros(6)
        for zg in p1.G2:
            v = p0.rt0_values(np.array([0.5]), np.array([0.5]), np.array([zg]), np.array([hx]), np.array([hy]),
                              np.array([hz]))[0, 0]
            th = cd["thB"][c] * (1 - zg) + cd["thT"][c] * zg
            want += 0.5 * prob.tau_theta * prob.dt * hx * hy * hz * v[:, 2] * dth / th
        np.testing.assert_allclose(one8 @ l1["q32"][c] @ E, want, rtol=1e-11, atol=1e-20)


@pytest.mark.parametrize("shape", [(2, 2, 2), (3, 2, 2)])
def test_hybrid_system_matches_dense_kkt(shape):
    prob, mesh = _mesh(*shape, perturb=0.05)
    loc = p1.local_matrices(mesh, prob)
    h = p1.HybridP1(mesh, loc)
    r_u, r_p = _rhs(mesh, 1)
    lam, u, p, _ = h.solve_direct(r_u, r_p)
    lam_d, u_d, p_d = h.solve_kkt_dense(r_u, r_p)
    np.testing.assert_allclose(lam, lam_d, rtol=1e-9, atol=1e-9 * np.abs(lam_d).max())
    np.testing.assert_allclose(u, u_d, rtol=1e-9, atol=1e-9 * np.abs(u_d).max())
    np.testing.assert_allclose(p, p_d, rtol=1e-9, atol=1e-9 * np.abs(p_d).max())


def test_hybrid_solution_equals_mixed_solution():
    """Horizontally homogeneous theta* (single valued on facets): the recovered broken (u, Pi)
    equals the continuous-RT1 mixed solution by sparse LU, which is also continuous in u . n."""
    prob, mesh = _mesh(3, 3, 3)
    loc = p1.local_matrices(mesh, prob)
    h = p1.HybridP1(mesh, loc)
    m = p1.MixedP1(mesh, loc)
    rng = np.random.default_rng(3)
    # a broken right-hand side that comes from a continuous one: r_u of a face dof is split equally
    # between the two cells (their outward signs differ), so both formulations pose the same problem
    sol_r = rng.standard_normal(m.nu + m.np_)
    full = np.where(m.full >= 0, sol_r[np.maximum(m.full, 0)], 0.0) * m.fsign
    shared = np.zeros_like(full)
    shared[:, : p1.NF] = 0.5
    shared[:, p1.NF:] = 1.0
    bnd = m.full < 0
    r = full * shared
    r[bnd] = 0.0
    r_u, r_p = r[:, : p1.NU], r[:, p1.NU:]
    lam, u, p, _ = h.solve_direct(r_u, r_p)
    um, pm = m.broken(m.solve(r_u, r_p))
    scale_u, scale_p = np.abs(um).max(), np.abs(pm).max()
    assert np.abs(u - um).max() <= 1e-9 * scale_u
    assert np.abs(p - pm).max() <= 1e-9 * scale_p


def test_recovered_velocity_is_continuous_and_vanishes_on_lid_and_ground():
    prob, mesh = _mesh(3, 2, 3, perturb=0.05)
    loc = p1.local_matrices(mesh, prob)
    h = p1.HybridP1(mesh, loc)
    r_u, r_p = _rhs(mesh, 5)
    lam, u, p, _ = h.solve_direct(r_u, r_p)
    flux = np.zeros(h.ntrace)
    np.add.at(flux, h.dofs.ravel(), u[:, : p1.NF].ravel())  # outward components of the two sides
    scale = np.abs(u[:, : p1.NF]).max()
    assert np.abs(flux).max() <= 1e-9 * scale
    bnd = np.repeat(mesh.boundary, 4)
    at_bnd = np.zeros(h.ntrace, bool)
    at_bnd[h.dofs.ravel()] = bnd[h.dofs.ravel()]
    for c in range(mesh.ncell):
        for f in (4, 5):
            if mesh.boundary[mesh.cell_faces[c, f]]:
                assert np.abs(u[c, 4 * f: 4 * f + 4]).max() <= 1e-9 * scale


def test_trace_operator_is_spd_in_the_symmetric_case():
    prob, mesh = _mesh(2, 2, 3, nbv=0.0)
    h = p1.HybridP1(mesh, p1.local_matrices(mesh, prob))
    S = h.S.toarray()
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    assert np.linalg.eigvalsh(0.5 * (S + S.T)).min() > 0.0


def _precond_problem(nx=4, ny=4, nlev=3, mg_levels=2, **kw):
    from oracle.problem import OracleProblem

    prob = make_box(nx=nx, ny=ny, nlev=nlev, dx=kw.pop("dx", 5e3), dz=250.0, mg_levels=mg_levels, **kw)
    mesh = BoxMesh(prob.nx, prob.ny, prob.nlev, prob.dx, prob.dy, prob.z)
    h = p1.HybridP1(mesh, p1.local_matrices(mesh, prob))
    H = OracleProblem(prob, with_precond=True).H
    return prob, mesh, h, H


def test_line_smoother_matrix_matches_dense_construction():
    prob, mesh, h, H = _precond_problem(3, 2, 3, mg_levels=1)
    S = h.S.toarray()
    n = S.shape[0]
    col_of = lambda T: (T // 4) % mesh.ncol if T // 4 < mesh.n_zface else -1  # noqa: E731
    D = np.zeros_like(S)
    for a in range(n):
        for b in range(n):
            za, zb = a // 4 < mesh.n_zface, b // 4 < mesh.n_zface
            if (za and zb and col_of(a) == col_of(b)) or (not za and a == b):
                D[a, b] = S[a, b]
    np.testing.assert_array_equal(p1.line_smoother_matrix(mesh, h.S).toarray(), D)
    # block tridiagonal with 4x4 blocks within a column: facets more than one level apart never couple
    for a, b in zip(*np.nonzero(D)):
        if a // 4 < mesh.n_zface:
            assert abs(a // 4 // mesh.ncol - b // 4 // mesh.ncol) <= 1


def test_gamma_and_prolongation():
    prob, mesh, h, H = _precond_problem(3, 2, 3, mg_levels=1)
    P = p1.trace_prolongation(mesh).toarray()
    assert np.allclose(P.sum(axis=1), 1.0)  # every dof is an average (one sided on lid/ground)
    tl = p1.TwoLevelP1(mesh, h.S, H, mg_levels=1)
    G = P.T @ h.S.toarray() @ P
    # both sums cancel strongly (row sums of H and S are small against their entries, as at order 0)
    np.testing.assert_allclose(tl.gamma, H.toarray().sum(axis=1) / G.sum(axis=1), rtol=1e-9)


def test_two_level_p1_is_linear_and_its_coarse_correction_helps():
    """M is a fixed linear map, and with the DG0 coarse correction FGMRES needs fewer iterations than
    with the LineSmooth sweeps alone.  (Unlike order 0, the cycle is not a contraction as a
    stationary iteration on this strongly anisotropic box: the DG0 space sees only cell averages of
    a p = 1 error; spectral radius of I - M S about 1.006 here, against 0.966 at order 0.)"""
    from oracle.krylov import fgmres

    prob, mesh, h, H = _precond_problem(4, 4, 4, mg_levels=2, perturb=0.05)
    tl = p1.TwoLevelP1(mesh, h.S, H, mg_levels=2)
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal(h.ntrace), rng.standard_normal(h.ntrace)
    np.testing.assert_allclose(tl(2.0 * a - 3.0 * b), 2.0 * tl(a) - 3.0 * tl(b), rtol=1e-9,
                               atol=1e-9 * np.abs(tl(a)).max())
    B = h.rhs(*_rhs(mesh, 9))
    smooth_only = lambda v: tl.line_smooth(np.zeros_like(v), v, tl.n_pre + tl.n_post)  # noqa: E731
    its_two = fgmres(lambda v: h.S @ v, tl, B, rtol=1e-10, restart=30, maxit=300)[2]
    its_smooth = fgmres(lambda v: h.S @ v, smooth_only, B, rtol=1e-10, restart=30, maxit=300)[2]
    assert its_two < 0.8 * its_smooth


def spla_solve(S, B):
    import scipy.sparse.linalg as spla

    return spla.splu(S.tocsc()).solve(B)


def test_fgmres_with_two_level_p1_reaches_the_direct_solution():
    from oracle.krylov import fgmres

    prob, mesh, h, H = _precond_problem(4, 4, 4, mg_levels=2, perturb=0.05)
    tl = p1.TwoLevelP1(mesh, h.S, H, mg_levels=2)
    r_u, r_p = _rhs(mesh, 9)
    B = h.rhs(r_u, r_p)
    x, hist, its, ok = fgmres(lambda v: h.S @ v, tl, B, rtol=1e-12, restart=30, maxit=200)
    lam = spla_solve(h.S, B)
    assert ok and its < 60
    assert np.abs(x - lam).max() <= 1e-9 * np.abs(lam).max()


def test_velocity_block_is_twelve_3x3_blocks():
    """On an axis-aligned cell the RT1 functions are Lagrange functions on the Gauss points in their
    tangential directions, which are orthogonal under the Gauss rule, so M = m2 - q22 couples a
    function only to the two others of its direction and tangential point: twelve 3x3 blocks
    {4 (2 d) + i, 4 (2 d + 1) + i, 24 + 4 d + i}.  The FP64 condensation of the library relies on it;
    checked on a stretched, perturbed box (every entry outside the blocks below 1e-14 of the largest)."""
    prob, mesh = _mesh(nx=3, ny=2, nlev=4, perturb=0.1, dx=6e3, ztop=9e3, stretch="quadratic")
    A = p1.local_matrices(mesh, prob)["A"]
    M = A[:, :36, :36]
    mask = np.zeros((36, 36), bool)
    for d in range(3):
        for i in range(4):
            idx = [8 * d + i, 8 * d + 4 + i, 24 + 4 * d + i]
            mask[np.ix_(idx, idx)] = True
    outside = np.abs(M[:, ~mask]).max()
    assert outside <= 1e-14 * np.abs(M).max(), outside
    # and the blocks themselves are full (no further structure assumed)
    assert np.abs(M[:, mask]).min() > 0
