"""Pins of the oracle's condensation, mixed solve and conservation (CPU only)."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.problem import OracleProblem, cells_from_soa
from synth import make_box, make_rhs

TINY = [
    dict(nx=3, ny=3, nlev=2, dx=10e3, dy=8e3, dz=1250.0, mg_levels=1, perturb=0.05),
    dict(nx=4, ny=4, nlev=3, dx=5e3, dy=5e3, dz=250.0, mg_levels=1, perturb=0.05),
    dict(nx=5, ny=3, nlev=4, dx=20e3, dy=10e3, ztop=30e3, stretch="quadratic", dt=1800.0, mg_levels=1),
]


@pytest.mark.parametrize("kw", TINY)
def test_condensed_equals_dense_kkt(kw):
    prob = make_box(**kw)
    o = OracleProblem(prob, with_precond=False)
    ruc, rpc = cells_from_soa(*make_rhs(prob, 3))
    lam, ub, pi, _ = o.hyb.solve_direct(ruc, rpc)
    lk, uk, pk = o.hyb.solve_kkt_dense(ruc, rpc)
    assert np.linalg.norm(lam - lk) <= 1e-11 * np.linalg.norm(lk)
    assert np.linalg.norm(ub - uk) <= 1e-11 * np.linalg.norm(uk)
    assert np.linalg.norm(pi - pk) <= 1e-11 * np.linalg.norm(pk)


@pytest.mark.parametrize("kw", TINY + [dict(nx=8, ny=6, nlev=5, dx=5e3, dz=250.0, mg_levels=1, perturb=0.1)])
def test_hybrid_equals_mixed_and_conserves(kw):
    prob = make_box(**kw)
    o = OracleProblem(prob, with_precond=False)
    ruc, rpc = cells_from_soa(*make_rhs(prob, 11))
    u, pi = o.mixed.solve(ruc, rpc)
    lam, ub, pih, _ = o.hyb.solve_direct(ruc, rpc)
    ubm = o.mixed.broken_from_continuous(u)
    assert np.linalg.norm(pih - pi) <= 1e-11 * np.linalg.norm(pi)
    assert np.linalg.norm(ub - ubm) <= 1e-11 * np.linalg.norm(ubm)
    mesh = o.mesh
    # continuity of normal flux: u_{K-,F} + u_{K+,F} = 0; zero flux through ground and lid
    flux = np.zeros(mesh.ntrace)
    np.add.at(flux, mesh.cell_faces.ravel(), ub.ravel())
    scale = np.abs(ub).max()
    assert np.abs(flux).max() <= 1e-11 * scale
    # discrete mass conservation: net outflow over the domain is zero
    assert abs(ub.sum()) <= 1e-11 * scale * mesh.ncell
    # mixed residual of the recovered hybrid solution
    uc = np.zeros(o.mixed.nu)
    for a in range(6):
        d = o.mixed.udof[mesh.cell_faces[:, a]]
        ok = d >= 0
        uc[d[ok]] = mesh.cell_sign[ok, a] * ub[ok, a]
    assert o.mixed.backward_error(uc, pih, ruc, rpc) <= 1e-12


def test_trace_operator_structure_and_symmetric_case():
    # symmetric special case: theta* constant (N = 0), no rotation -> S symmetric positive definite
    prob = make_box(nx=4, ny=3, nlev=4, dx=10e3, dy=6e3, dz=1000.0, nbv=0.0, mg_levels=1)
    o = OracleProblem(prob, with_precond=False)
    S = o.hyb.S.toarray()
    assert np.abs(S - S.T).max() <= 1e-14 * np.abs(S).max()
    np.linalg.cholesky(S)
    # general state: mildly nonsymmetric; 11 entries per interior row, 6 on ground/lid rows
    prob = make_box(nx=4, ny=4, nlev=4, dx=10e3, dz=1000.0, mg_levels=1)
    o = OracleProblem(prob, with_precond=False)
    nnz = np.diff(o.hyb.S.indptr)
    bnd = o.mesh.boundary
    assert set(nnz[bnd]) == {6}
    assert set(nnz[~bnd]) == {11}
    # S^zz is tridiagonal per column
    Sz = o.hyb.S[: o.mesh.n_zface, : o.mesh.n_zface].tocoo()
    same = (Sz.row % o.mesh.ncol) == (Sz.col % o.mesh.ncol)
    assert np.all(np.abs(Sz.row[same] - Sz.col[same]) // o.mesh.ncol <= 1)
    assert not np.any(same == False)  # noqa: E712  (no z-z coupling across columns)
    ev = np.linalg.eigvals(o.hyb.S.toarray())
    assert ev.real.min() > 0


def test_direct_trace_solve_residual():
    prob = make_box(nx=6, ny=6, nlev=5, dx=5e3, dz=250.0, mg_levels=1)
    o = OracleProblem(prob, with_precond=False)
    ruc, rpc = cells_from_soa(*make_rhs(prob, 0))
    lam, _, _, B = o.hyb.solve_direct(ruc, rpc)
    assert np.linalg.norm(B - o.hyb.S @ lam) <= 1e-12 * np.linalg.norm(B)
    lu = spla.splu(o.hyb.S.tocsc())
    np.testing.assert_allclose(lu.solve(B), lam, rtol=0, atol=1e-12 * np.abs(lam).max())


def test_all_rows_residuals_match_the_assembled_operators():
    """The chunked all-rows residuals (used at sizes the assembled operators do not fit) equal
    the assembled ones on a small box: ||B - S lambda|| / ||B||, the continuity defect C^T X
    (= B - S lambda for the recovered X) and the componentwise backward error of the 2x2 system."""
    from oracle.allrows import all_rows
    from oracle.local import local_matrices
    from oracle.problem import OracleProblem, cells_from_soa
    from synth import make_box, make_rhs

    prob = make_box(nx=6, ny=4, nlev=5, dx=8e3, dz=600.0, mg_levels=1, perturb=0.05)
    o = OracleProblem(prob, with_precond=False)
    ruc, rpc = cells_from_soa(*make_rhs(prob, 3))
    lam_ref, _, _, B = o.hyb.solve_direct(ruc, rpc)
    lam = lam_ref + 1e-6 * np.random.default_rng(4).standard_normal(lam_ref.shape) * np.abs(lam_ref).max()
    ub, pi = o.hyb.recover(lam, ruc, rpc)
    res = all_rows(lambda cells: local_matrices(o.mesh, prob, cells=cells), o.mesh, ruc, rpc,
                   [(lam, ub, pi)], chunk=37)[0]
    tr = np.linalg.norm(B - o.hyb.S @ lam) / np.linalg.norm(B)
    assert abs(res["trace_res"] - tr) <= 1e-9 * tr
    # C^T X of the recovery is B - S lambda (Sec. 2.4)
    assert abs(res["defect_norm"] - tr) <= 1e-6 * tr
    u = np.zeros(o.mixed.nu)
    cnt = np.zeros(o.mixed.nu)
    for a in range(6):
        d = o.mixed.udof[o.mesh.cell_faces[:, a]]
        ok = d >= 0
        np.add.at(u, d[ok], o.mesh.cell_sign[ok, a] * ub[ok, a])
        np.add.at(cnt, d[ok], 1.0)
    berr = o.mixed.backward_error(u / cnt, pi, ruc, rpc)
    assert abs(res["mixed_berr"] - berr) <= 1e-9 * berr
    # every cell satisfies its own equations at its recovered fluxes, so the 2x2 residual is the
    # continuity defect's doing: the backward error stays under what |M| |x - X| allows; a wrong
    # recovered Pi breaks that
    assert berr <= res["mixed_berr_bound"] + 1e-13
    ub0, pi0 = o.hyb.recover(lam_ref, ruc, rpc)
    good, bad = all_rows(lambda cells: local_matrices(o.mesh, prob, cells=cells), o.mesh, ruc, rpc,
                         [(lam_ref, ub0, pi0), (lam_ref, ub0, pi0 * (1 + 1e-6))], chunk=37)
    assert good["mixed_berr"] <= good["mixed_berr_bound"] + 1e-13
    assert bad["mixed_berr"] > 10 * bad["mixed_berr_bound"]
