"""Pins of the oracle's preconditioner and Krylov solver (CPU only)."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.krylov import fgmres
from oracle.precond import PressureMultigrid, trace_prolongation
from oracle.problem import OracleProblem, cells_from_soa
from synth import make_box, make_rhs


@pytest.fixture(scope="module")
def box():
    prob = make_box(nx=8, ny=8, nlev=6, dx=10e3, dy=8e3, dz=1250.0, mg_levels=3, perturb=0.05)
    return prob, OracleProblem(prob)


def test_pressure_operator_row_sums_and_stencil(box):
    prob, o = box
    H = o.H
    # the discrete gradient G annihilates constants (volume and facet terms cancel), so H 1 = M3^Pi 1
    ones = np.ones(H.shape[0])
    np.testing.assert_allclose(H @ ones, o.mixed.M3pi.diagonal(), rtol=1e-9, atol=0)
    np.testing.assert_allclose(o.mixed.G @ ones, 0.0, atol=1e-9 * np.abs(o.mixed.G).max())
    # 7-point stencil on every level, off-diagonals negative; coarse operators keep the row sums
    mg = o.pc.mg
    for lev, Hl in enumerate(mg.H):
        assert np.diff(Hl.indptr).max() <= 7
        off = Hl - sp.diags(Hl.diagonal())
        assert off.data.max() < 0
        if lev:
            P = mg.P[lev - 1]
            np.testing.assert_allclose(Hl @ np.ones(Hl.shape[0]), P.T @ (mg.H[lev - 1] @ np.ones(P.shape[0])), rtol=1e-9)
    # lumped mass: every entry positive
    from oracle.precond import lumped_velocity_mass

    assert lumped_velocity_mass(o.mixed).min() > 0


def test_line_smoother_exact_when_columns_decouple():
    """As dx -> infinity the horizontal couplings vanish and one sweep with omega = 1 solves the z part."""
    errs = []
    for dx in (1e6, 1e8):
        prob = make_box(nx=4, ny=4, nlev=5, dx=dx, dz=1000.0, mg_levels=1)
        o = OracleProblem(prob)
        ruc, rpc = cells_from_soa(*make_rhs(prob, 0))
        lam, _, _, B = o.hyb.solve_direct(ruc, rpc)
        o.pc.omega = 1.0
        l1 = o.pc.line_smooth(np.zeros_like(B), B, 1)
        nz = o.mesh.n_zface
        errs.append(np.linalg.norm(l1[:nz] - lam[:nz]) / np.linalg.norm(lam[:nz]))
    assert errs[1] < 1e-4 and errs[1] < 1e-2 * errs[0]


def test_smoother_sign_reading():
    """With the update lambda - omega*delta the sweep diverges; with + it contracts for omega <= 0.8
    and diverges beyond, matching the stability limit reported for omega > 0.8."""
    prob = make_box(nx=6, ny=6, nlev=4, dx=10e3, dz=1250.0, mg_levels=1)
    o = OracleProblem(prob)
    S, D = o.hyb.S.toarray(), o.pc.D.toarray()
    DinvS = np.linalg.solve(D, S)
    rho = lambda sgn, om: np.abs(np.linalg.eigvals(np.eye(len(S)) - sgn * om * DinvS)).max()  # noqa: E731
    assert rho(-1, 0.6) > 2.0
    assert rho(+1, 0.6) < 1.0
    assert rho(+1, 0.8) < 1.0
    assert rho(+1, 1.0) > 1.0


def test_vcycle_and_two_level_contract(box):
    prob, o = box
    rng = np.random.default_rng(5)
    H = o.H
    b = rng.standard_normal(H.shape[0])
    x = np.zeros_like(b)
    r0 = np.linalg.norm(b)
    for _ in range(6):
        x = x + o.pc.mg.vcycle(b - H @ x)
    assert np.linalg.norm(b - H @ x) < 0.1 * r0
    # when the horizontal coupling vanishes (dx -> infinity) H_z = H and one sweep with omega = 1 is exact
    wide = make_box(nx=4, ny=4, nlev=6, dx=1e11, dz=1250.0, mg_levels=1)
    ow = OracleProblem(wide)
    bw = rng.standard_normal(ow.H.shape[0])
    mg1 = PressureMultigrid(ow.H, 4, 4, 6, levels=1, omega=1.0, coarse_sweeps=1, coarse_cheb=None)
    y = mg1.vcycle(bw)
    assert np.linalg.norm(bw - ow.H @ y) < 1e-10 * np.linalg.norm(bw)
    # the two-level cycle is a linear map
    B1, B2 = rng.standard_normal(o.mesh.ntrace), rng.standard_normal(o.mesh.ntrace)
    np.testing.assert_allclose(o.pc(2.0 * B1 - 3.0 * B2), 2.0 * o.pc(B1) - 3.0 * o.pc(B2), rtol=1e-10,
                               atol=1e-12 * np.abs(o.pc(B1)).max())
    # as a stationary iteration on S it converges
    S = o.hyb.S
    lam = np.zeros_like(B1)
    for _ in range(15):
        lam = lam + o.pc(B1 - S @ lam)
    assert np.linalg.norm(B1 - S @ lam) < 0.1 * np.linalg.norm(B1)


def test_gamma_against_dense_products(box):
    prob, o = box
    P = trace_prolongation(o.mesh).toarray()
    # P maps a constant to a constant (one-sided on lid/ground facets)
    np.testing.assert_allclose(P @ np.ones(P.shape[1]), 1.0)
    S = o.hyb.S.toarray()
    HG = P.T @ S @ P
    gamma = o.H.toarray().sum(axis=1) / HG.sum(axis=1)
    np.testing.assert_allclose(o.pc.gamma, gamma, rtol=1e-9)
    assert o.pc.gamma.min() > 0


def test_fgmres_minimal_residual_property():
    rng = np.random.default_rng(0)
    n = 40
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n)
    Mmat = np.diag(1.0 / np.diag(A))
    for k in (1, 3, 7):
        x, hist, its, conv = fgmres(lambda v: A @ v, lambda v: Mmat @ v, b, rtol=0.0, restart=50, maxit=k)
        # brute force: minimise ||b - A M y|| over the Krylov space of A M
        AM = A @ Mmat
        K = np.stack([np.linalg.matrix_power(AM, i) @ b for i in range(k)], axis=1)
        y, *_ = np.linalg.lstsq(AM @ K, b, rcond=None)
        best = np.linalg.norm(b - AM @ K @ y)
        assert abs(np.linalg.norm(b - A @ x) - best) <= 1e-10 * np.linalg.norm(b)
        assert abs(hist[-1] * np.linalg.norm(b) - best) <= 1e-10 * np.linalg.norm(b)


def test_preconditioned_solve_reaches_tolerance(box):
    prob, o = box
    ruc, rpc = cells_from_soa(*make_rhs(prob, 2))
    B = o.hyb.rhs(ruc, rpc)
    x, hist, its, conv = o.solve_fgmres(B, rtol=1e-10)
    assert conv and its < 40
    assert np.linalg.norm(B - o.hyb.S @ x) <= 1e-10 * np.linalg.norm(B) * 1.01
    assert all(h2 <= h1 * (1 + 1e-12) for h1, h2 in zip(hist, hist[1:]))
    xu, hu, itu, cu = o.solve_fgmres(B, rtol=1e-10, precondition=False, maxit=2000)
    assert itu > 2 * its


def test_chebyshev_semi_iteration_closed_form():
    """After d steps from x = 0 the error of the Chebyshev semi-iteration is p_d(M^-1 A) x with
    p_d(t) = T_d((theta - t) / delta) / T_d(theta / delta): checked on a diagonal A (M = I) with
    eigenvalues inside and outside the interval, T_d from numpy's Chebyshev series."""
    from numpy.polynomial import chebyshev as C

    from oracle.precond import chebyshev_solve

    rng = np.random.default_rng(3)
    lam = np.concatenate([np.linspace(0.02, 2.0, 9), [0.005, 0.5, 1.3, 2.2]])
    x_true = rng.standard_normal(lam.size)
    b = lam * x_true
    lo, hi = 0.02, 2.0
    theta, delta = (hi + lo) / 2, (hi - lo) / 2
    for d in (1, 2, 3, 6, 11):
        x = chebyshev_solve(lambda v: lam * v, lambda v: v, b, d, lo, hi)
        Td = C.Chebyshev.basis(d)
        p = Td((theta - lam) / delta) / Td(theta / delta)
        np.testing.assert_allclose(x_true - x, p * x_true, rtol=1e-10, atol=1e-12)
        # inside the interval the error factor is at most 1 / T_d(theta / delta)
        inside = (lam >= lo) & (lam <= hi)
        assert np.all(np.abs(p[inside]) <= 1.0 / Td(theta / delta) * (1 + 1e-12))


def test_chebyshev_coarsest_solve(box):
    """The eigenvalues of H_z^-1 H lie in (0, 2) on every level (the upper end of the default
    interval), and with the exact interval and enough steps the Chebyshev coarsest solve reaches
    the direct solution within its error bound."""
    from numpy.polynomial import chebyshev as C

    from oracle.precond import chebyshev_solve

    prob, o = box
    mg = o.pc.mg
    for lev in range(mg.nlevels):
        Hd, Hz = mg.H[lev].toarray(), mg.Hz[lev].toarray()
        ev = np.linalg.eigvals(np.linalg.solve(Hz, Hd)).real
        assert ev.min() > 0 and ev.max() < 2.0, (lev, ev.min(), ev.max())
    L = mg.nlevels - 1
    Hd, Hz = mg.H[L].toarray(), mg.Hz[L].toarray()
    ev = np.linalg.eigvals(np.linalg.solve(Hz, Hd)).real
    lo, hi = ev.min(), ev.max()
    rng = np.random.default_rng(8)
    b = rng.standard_normal(Hd.shape[0])
    x_ref = np.linalg.solve(Hd, b)
    d = 40
    x = chebyshev_solve(lambda v: mg.H[L] @ v, mg.Hz_lu[L].solve, b, d, lo, hi)
    theta, delta = (hi + lo) / 2, (hi - lo) / 2
    bound = 1.0 / C.Chebyshev.basis(d)(theta / delta)
    # error in the H-norm (H_z^-1 H is self-adjoint there) shrinks by at most the bound
    e, e0 = x_ref - x, x_ref
    assert np.sqrt(e @ Hd @ e) <= bound * np.sqrt(e0 @ Hd @ e0) * (1 + 1e-8)


def test_single_level_configuration():
    """The paper's hybridised single-level configuration: the preconditioner is LineSmooth alone.
    One sweep from zero is omega D^-1 B (D: the column blocks of S^zz and diag(S^hh)); two sweeps
    add omega D^-1 of the new residual; FGMRES needs more iterations with it than with the
    two-level cycle, and fewer with more sweeps (the paper's ordering of its configurations)."""
    import scipy.sparse.linalg as spla

    from oracle.precond import line_smoother_matrix
    from oracle.problem import OracleProblem, cells_from_soa
    from synth import make_box, make_rhs

    prob = make_box(nx=12, ny=12, nlev=8, dx=10e3, dz=1250.0, mg_levels=3)
    o1 = OracleProblem(prob, n_pre=1, n_post=0, coarse=False)
    S = o1.hyb.S
    D = line_smoother_matrix(o1.mesh, S).tocsc()
    B = cells_from_soa(*make_rhs(prob, 0))
    B = o1.hyb.rhs(*B)
    z1 = spla.spsolve(D, B) * 0.6
    np.testing.assert_allclose(o1.pc(B), z1, rtol=1e-12, atol=1e-12 * np.abs(z1).max())
    o2 = OracleProblem(prob, n_pre=1, n_post=1, coarse=False)
    z2 = z1 + 0.6 * spla.spsolve(D, B - S @ z1)
    np.testing.assert_allclose(o2.pc(B), z2, rtol=1e-11, atol=1e-12 * np.abs(z2).max())
    its = {}
    for n in (1, 3):
        o = OracleProblem(prob, n_pre=n, n_post=0, coarse=False)
        its[n] = o.solve_fgmres(B, rtol=1e-8, maxit=2000)[2]
    its["3c"] = OracleProblem(prob).solve_fgmres(B, rtol=1e-8)[2]
    assert its["3c"] < its[3] < its[1]


def test_line_smooth_error_propagation():
    """k LineSmooth sweeps from zero are a preconditioner M_k with I - M_k S = (I - omega D^-1 S)^k
    (Alg. 1 is a damped block-Jacobi iteration).  Consequences the solver-parameter study relies on:
    one sweep is omega D^-1, a scalar multiple of a fixed map, so FGMRES takes the same iterations
    for every omega; and where omega mu > 2 for an eigenvalue mu of D^-1 S, an even k makes the
    eigenvalue 1 - (1 - omega mu)^k of M_k S negative (an indefinite preconditioned operator)."""
    import scipy.sparse.linalg as spla

    from oracle.precond import line_smoother_matrix
    from oracle.problem import OracleProblem, cells_from_soa
    from synth import make_box, make_rhs

    prob = make_box(nx=8, ny=8, nlev=8, dx=10e3, dz=1250.0, mg_levels=2, perturb=0.05)
    x = np.random.default_rng(9).standard_normal(OracleProblem(prob, with_precond=False).mesh.ntrace)
    for om in (0.6, 0.9):
        for k in (1, 2, 3):
            o = OracleProblem(prob, omega=om, n_pre=k, n_post=0, coarse=False)
            S = o.hyb.S
            lu = spla.splu(line_smoother_matrix(o.mesh, S).tocsc())
            e = x.copy()
            for _ in range(k):
                e = e - om * lu.solve(S @ e)
            np.testing.assert_allclose(x - o.pc(S @ x), e, rtol=1e-10, atol=1e-10 * np.abs(x).max())
    B = cells_from_soa(*make_rhs(prob, 0))
    its = []
    for om in (0.3, 0.9):
        o = OracleProblem(prob, omega=om, n_pre=1, n_post=0, coarse=False)
        its.append(o.solve_fgmres(o.hyb.rhs(*B), rtol=1e-8, maxit=2000)[2])
    assert its[0] == its[1]
    mu = np.linalg.eigvals(spla.splu(line_smoother_matrix(o.mesh, S).tocsc()).solve(S.toarray())).real
    om = 2.2 / mu.max()
    lam2 = 1.0 - (1.0 - om * mu) ** 2
    assert lam2.min() < 0 < lam2.max()
    lam3 = 1.0 - (1.0 - om * mu) ** 3
    assert lam3.min() > 0


def test_bicgstab_and_krylov_coarse_solve():
    """BiCGStab reaches its tolerance and the sparse direct solution; with the exact inverse as the
    preconditioner it stops after one half step; the two-level cycle with the coarse system solved
    to 1e-14 by BiCGStab + V-cycle (the paper's Configuration 3a) is the cycle with an exact coarse
    solve, and 1e-2 (3b) leaves at most that coarse residual."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    from oracle.krylov import bicgstab
    from oracle.problem import OracleProblem, cells_from_soa
    from synth import make_box, make_rhs

    rng = np.random.default_rng(5)
    n = 60
    A = sp.random(n, n, density=0.1, random_state=5) + sp.diags(4.0 + rng.random(n))
    A = A.tocsr()
    b = rng.standard_normal(n)
    xd = spla.spsolve(A.tocsc(), b)
    x = bicgstab(lambda v: A @ v, lambda v: v, b, 1e-12)
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    lu = spla.splu(A.tocsc())
    calls = []
    x1 = bicgstab(lambda v: (calls.append(1), A @ v)[1], lu.solve, b, 1e-12)
    assert len(calls) == 1 and np.linalg.norm(x1 - xd) <= 1e-12 * np.linalg.norm(xd)

    prob = make_box(nx=12, ny=12, nlev=8, dx=10e3, dz=1250.0, mg_levels=3, perturb=0.05)
    o = OracleProblem(prob)
    B = o.hyb.rhs(*cells_from_soa(*make_rhs(prob, 1)))
    pc = o.pc
    lam = pc.line_smooth(np.zeros_like(B), B, pc.n_pre)
    Bbar = pc.gamma * (pc.P.T @ (B - pc.S @ lam))
    H0 = pc.mg.H[0]
    zexact = pc.line_smooth(lam + pc.P @ spla.spsolve(H0.tocsc(), Bbar), B, pc.n_post)
    o3a = OracleProblem(prob, coarse=("bicgstab", 1e-14))
    np.testing.assert_allclose(o3a.pc(B), zexact, rtol=0, atol=1e-10 * np.abs(zexact).max())
    dpi = bicgstab(lambda v: H0 @ v, pc.mg.vcycle, Bbar, 1e-2)
    assert np.linalg.norm(Bbar - H0 @ dpi) <= 1e-2 * np.linalg.norm(Bbar)


def _lumped_closed_form(prob, mesh):
    """Sec. 2.3 lumping on an axis-aligned box, worked out from the App. A cell matrices: each cell
    adds (1/3 + 1/6) a of its velocity block to the row of a facet it shares (the -1/6 coupling to
    the opposite facet changes sign with the global orientation), so a vertical x / y facet gets
    a_x / a_y and an interior horizontal facet (1 + beta) a_z / 2 from each of its two cells (the
    row sum runs over the kept dofs: the ground and lid facets have none)."""
    L, ncol = mesh.nlev, mesh.ncol
    hx, hy, hz = mesh.dx, mesh.dy, mesh.dz
    th, pih = prob.theta_w, prob.exner_hat_w
    beta = -prob.tau_u * prob.tau_theta * prob.dt**2 * prob.cp * (pih[1:] - pih[:-1]) * (th[1:] - th[:-1]) / hz[:, None] ** 2
    az = (1.0 + beta) * (hz / (hx * hy))[:, None]  # [L][ncol]
    # a cell's share of its top (bottom) facet row is az / 2, or az / 3 when its other horizontal
    # facet is the ground (lid): that facet has no velocity dof, so its -1/6 coupling drops out
    share_top = az / 2.0
    share_bot = az / 2.0
    share_top[0] = az[0] / 3.0
    share_bot[L - 1] = az[L - 1] / 3.0
    m2 = np.full(mesh.ntrace, np.nan)
    m2[ncol:L * ncol] = (share_top[:-1] + share_bot[1:]).ravel()  # interior horizontal facets k = 1..L-1
    ax = hx / (hy * hz)
    ay = hy / (hx * hz)
    for k in range(L):
        base = mesh.n_zface + k * 2 * ncol
        m2[base:base + ncol] = ax[k]
        m2[base + ncol:base + 2 * ncol] = ay[k]
    return m2


@pytest.mark.parametrize(
    "kw",
    [
        dict(nx=4, ny=3, nlev=5, dx=10e3, dy=7e3, dz=800.0, mg_levels=1),
        dict(nx=3, ny=4, nlev=6, dx=5e3, dy=6e3, ztop=30e3, stretch="quadratic", mg_levels=1, perturb=0.1),
    ],
)
def test_lumped_mass_and_pressure_operator_closed_forms(kw):
    """The lumped velocity mass and every entry of H = -B M2l^-1 G + M3^Pi against closed forms
    of Sec. 2.3 and App. A; the same lumping done in outward (broken) orientation fails."""
    from oracle.mixed import MixedSystem
    from oracle.local import local_matrices
    from oracle.mesh import BoxMesh
    from oracle.precond import lumped_velocity_mass, pressure_operator

    prob = make_box(**kw)
    mesh = BoxMesh(prob.nx, prob.ny, prob.nlev, prob.dx, prob.dy, prob.z)
    loc = local_matrices(mesh, prob)
    mixed = MixedSystem(mesh, loc, prob)
    ref = _lumped_closed_form(prob, mesh)
    interior = ~mesh.boundary
    got = lumped_velocity_mass(mixed)
    np.testing.assert_allclose(got, ref[interior], rtol=1e-12, atol=0)

    # H entry by entry.  Facet F of cells K- (normal leaves) and K+: H[K-, K+] = d^{K-}_F k_F / m2(F)
    # with the sign pattern of B (outward d) and G (outward g = -k), and
    # H[K, K] = m_K + sum over non-boundary facets of d^K_F k_F / m2(F).
    L, ncol, nx = mesh.nlev, mesh.ncol, mesh.nx
    tr, tu, dt, cp = prob.tau_rho, prob.tau_u, prob.dt, prob.cp
    th = prob.theta_w
    q = prob.tau_theta * dt * (th[1:] - th[:-1]) / (th[1:] + th[:-1])  # [L][ncol]
    m_k = (1 - prob.kappa) / prob.kappa * (mesh.dx * mesh.dy * mesh.dz)[:, None] / prob.exner_c
    kbar = tu * dt * cp * 0.5 * (th[1:] + th[:-1])  # k on the vertical facets of layer k
    Href = np.zeros((mesh.ncell, mesh.ncell))
    cell = lambda k, ix, iy: k * ncol + (iy % mesh.ny) * nx + (ix % nx)  # noqa: E731
    for k in range(L):
        for iy in range(mesh.ny):
            for ix in range(nx):
                c = cell(k, ix, iy)
                col = iy * nx + ix
                diag = m_k[k, col]
                for dxy, fn, m2f in (((1, 0), mesh.xface, None), ((0, 1), mesh.yface, None)):
                    # the facet on the E / N side of this cell, shared with the next column
                    f = fn(k, ix + dxy[0], iy + dxy[1])
                    other = cell(k, ix + dxy[0], iy + dxy[1])
                    coup = -tr * dt * kbar[k, col] / ref[f]
                    Href[c, other] += coup
                    Href[other, c] += coup
                    diag += tr * dt * kbar[k, col] / ref[f]
                    diag += tr * dt * kbar[k, col] / ref[fn(k, ix, iy)]
                if k + 1 < L:  # interior horizontal facet above: K- = this cell, K+ = the one above
                    f = mesh.zface(k + 1, ix, iy)
                    up = cell(k + 1, ix, iy)
                    kf = tu * dt * cp * th[k + 1, col]
                    Href[c, up] += -(tr * dt + q[k, col]) * kf / ref[f]
                    Href[up, c] += -(tr * dt - q[k + 1, col]) * kf / ref[f]
                    diag += (tr * dt + q[k, col]) * kf / ref[f]
                if k > 0:
                    f = mesh.zface(k, ix, iy)
                    kf = tu * dt * cp * th[k, col]
                    diag += (tr * dt - q[k, col]) * kf / ref[f]
                Href[c, c] += diag
    H = pressure_operator(mixed).toarray()
    np.testing.assert_allclose(H, Href, rtol=1e-11, atol=1e-12 * np.abs(Href).max())

    # a plausible mistake: lumping the broken (outward-oriented) cell blocks without the sign map
    # gives positive values a third as large on uniform cells, and H's couplings three times larger
    wrong = np.zeros(mesh.ntrace)
    for a in range(6):
        for b in range(6):
            np.add.at(wrong, mesh.cell_faces[:, a], loc["A"][:, a, b])
    wrong = wrong[interior]
    assert wrong.min() > 0  # it would pass a positivity pin
    assert np.abs(wrong / ref[interior] - 1.0).min() > 0.5
    Hwrong = pressure_operator(mixed, wrong).toarray()
    assert np.abs(Hwrong - Href).max() > 0.5 * np.abs(Href - np.diag(np.diag(Href))).max()


def test_patch_cached_line_smoother():
    """The Sec. 4.2 variant caching the column matrices over patches of columns (here the 2x2 patches
    of the first coarsening): on a horizontally homogeneous box every column has the same S^zz and
    the smoother is unchanged; with cell-to-cell variation every column's block is the patch mean
    (checked for one patch entry by entry from S); FGMRES with it still reaches the tolerance."""
    from oracle.precond import line_smoother_matrix

    prob = make_box(nx=8, ny=8, nlev=5, dx=10e3, dz=800.0, mg_levels=2)
    o = OracleProblem(prob)
    patch = prob.levels[1].parent
    D0 = line_smoother_matrix(o.mesh, o.hyb.S)
    Dp = line_smoother_matrix(o.mesh, o.hyb.S, patch)
    assert abs(Dp - D0).max() <= 1e-12 * abs(D0).max()
    prob = make_box(nx=8, ny=8, nlev=5, dx=10e3, dz=800.0, mg_levels=2, perturb=0.2)
    o = OracleProblem(prob)
    patch = prob.levels[1].parent
    S = o.hyb.S.tocsr()
    D0 = line_smoother_matrix(o.mesh, S)
    Dp = line_smoother_matrix(o.mesh, S, patch)
    assert abs(Dp - D0).max() > 1e-6 * abs(D0).max()
    ncol = o.mesh.ncol
    members = np.nonzero(patch == patch[9])[0]
    assert members.size == 4
    for k in range(1, o.mesh.nlev):
        for dk in (-1, 0, 1):
            ref = np.mean([S[k * ncol + c, (k + dk) * ncol + c] for c in members])
            for c in members:
                assert abs(Dp[k * ncol + c, (k + dk) * ncol + c] - ref) <= 1e-13 * abs(ref)
    # vertical-facet rows keep their own diagonal
    h = o.mesh.n_zface + 3
    assert Dp[h, h] == S[h, h]
    ruc, rpc = cells_from_soa(*make_rhs(prob, 0))
    B = o.hyb.rhs(ruc, rpc)
    _, hist0, its0, conv0 = o.solve_fgmres(B, rtol=1e-8)
    op = OracleProblem(prob, smoother_patch=True)
    _, histp, itsp, convp = op.solve_fgmres(B, rtol=1e-8)
    assert conv0 and convp and itsp <= its0 + 3
