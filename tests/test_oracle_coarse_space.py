"""Oracle coarse-space devices (CPU): the conforming vertex (Q1) coarse space of Sec. 4.2, the
agglomerated cell spaces of the pressure multigrid's levels, and the exact Galerkin corrections that
bound what a coarse space, or a correction stage after the coarse correction of Alg. 2, can give.

The prolongations are pinned by geometry (a linear function's facet means are its values at the
facet centres), the corrections by their defining properties (an exact solve when the coarse space
is the whole trace space, Galerkin orthogonality of the corrected residual).  The iteration counts
recorded at the end are measurements on a small box of the benchmark's physics: they back the
statements that the Q1 coarse space cuts no iteration that DG0 does not, and that a correction
confined to 2x2 or 4x4 agglomerated cells gains less than one on the fine cells."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.krylov import fgmres
from oracle.precond import (BestCorrectionAfter, GalerkinTwoLevel, agglomerated_cell_injection,
                            vertex_trace_prolongation)
from oracle.problem import OracleProblem, cells_from_soa
from synth import make_box, make_rhs


@pytest.fixture(scope="module")
def box():
    prob = make_box(nx=8, ny=8, nlev=32, dx=5e3, dz=250.0, dt=600.0, mg_levels=3)
    o = OracleProblem(prob, with_mixed=False)
    return prob, o


@pytest.fixture(scope="module")
def tiny():
    prob = make_box(nx=4, ny=4, nlev=4, dx=5e3, dz=250.0, dt=600.0, mg_levels=2)
    return prob, OracleProblem(prob, with_mixed=False)


def test_vertex_prolongation_reproduces_linear_functions(box):
    prob, o = box
    m = o.mesh
    Pv = vertex_trace_prolongation(m)
    assert Pv.shape == (m.ntrace, m.ncol * (m.nlev + 1))
    assert np.allclose(np.asarray(Pv.sum(axis=1)).ravel(), 1.0)
    assert np.all(np.diff(Pv.indptr) == 4)
    # f = 1 + 2x + 3y + 5z on the vertices; its facet means are its values at the facet centres,
    # on every facet whose corners do not wrap round the periodic edge
    nx, ny, L = m.nx, m.ny, m.nlev
    k, iy, ix = np.meshgrid(np.arange(L + 1), np.arange(ny), np.arange(nx), indexing="ij")
    f = lambda x, y, z: 1.0 + 2.0 * x / m.dx + 3.0 * y / m.dy + 5.0 * z / 1e3
    lam = Pv @ f(ix * m.dx, iy * m.dy, m.z[k]).ravel()
    zc = 0.5 * (m.z[:-1] + m.z[1:])
    for kk in (0, 5, L - 1):
        for jy in (0, 3, ny - 2):
            for jx in (0, 2, nx - 2):
                assert lam[m.zface(kk, jx, jy)] == pytest.approx(f((jx + .5) * m.dx, (jy + .5) * m.dy, m.z[kk]))
                assert lam[m.xface(kk, jx, jy)] == pytest.approx(f(jx * m.dx, (jy + .5) * m.dy, zc[kk]))
                assert lam[m.yface(kk, jx, jy)] == pytest.approx(f((jx + .5) * m.dx, jy * m.dy, zc[kk]))


def test_agglomerated_injection_partitions_the_cells(box):
    prob, o = box
    pars = [lv.parent for lv in prob.levels[1:]]
    for l in (1, 2):
        Q = agglomerated_cell_injection(o.mesh, pars[:l])
        assert np.all(np.diff(Q.indptr) == 1)  # every fine cell in exactly one coarse cell
        sizes = np.asarray(Q.sum(axis=0)).ravel()
        assert np.all(sizes == 4 ** l)
        # no vertical coarsening: a coarse cell's children share one layer
        rows, cols = Q.nonzero()
        ncl = Q.shape[1] // o.mesh.nlev
        assert np.array_equal(rows // o.mesh.ncol, cols // ncl)


def test_whole_space_corrections_are_exact_solves(tiny):
    prob, o = tiny
    S = o.hyb.S
    I = sp.identity(S.shape[0], format="csr")
    B = np.random.default_rng(3).standard_normal(S.shape[0])
    x = np.linalg.solve(S.toarray(), B)
    assert np.allclose(GalerkinTwoLevel(o.pc, I)(B), x, rtol=0, atol=1e-10 * np.abs(x).max())
    assert np.allclose(BestCorrectionAfter(o.pc, S, I)(B), x, rtol=0, atol=1e-10 * np.abs(x).max())


def test_corrections_are_galerkin_orthogonal(tiny):
    prob, o = tiny
    S = o.hyb.S
    B = np.random.default_rng(4).standard_normal(S.shape[0])
    for Pc in (o.pc.P, vertex_trace_prolongation(o.mesh)):
        z = BestCorrectionAfter(o.pc, S, Pc)(B)
        r = Pc.T @ (B - S @ z)
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(Pc.T @ B)
        # the two-level form: orthogonal after its coarse step, before the post-smoothing
        g = GalerkinTwoLevel(o.pc, Pc)
        lam = o.pc.line_smooth(np.zeros_like(B), B, o.pc.n_pre)
        lam = lam + g.Pc @ g.lu.solve(g.Pc.T @ (B - S @ lam))
        assert np.linalg.norm(Pc.T @ (B - S @ lam)) <= 1e-10 * np.linalg.norm(Pc.T @ B)


def _its(o, M, seed=1):
    prob = o.prob
    B = o.hyb.rhs(*cells_from_soa(*make_rhs(prob, seed)))
    _, _, it, ok = fgmres(lambda x: o.hyb.S @ x, M, B, rtol=1e-8)
    assert ok
    return it


def test_conforming_coarse_space_gains_nothing_over_dg0(box):
    prob, o = box
    paper = _its(o, o.pc)
    dg0 = _its(o, GalerkinTwoLevel(o.pc, o.pc.P))
    q1 = _its(o, GalerkinTwoLevel(o.pc, vertex_trace_prolongation(o.mesh)))
    # measured: 14, 9, 10
    assert dg0 < paper and q1 < paper
    assert q1 >= dg0


def test_coarser_correction_spaces_gain_less(box):
    prob, o = box
    pars = [lv.parent for lv in prob.levels[1:]]
    paper = _its(o, o.pc)
    its = [_its(o, BestCorrectionAfter(o.pc, o.hyb.S, o.pc.P @ agglomerated_cell_injection(o.mesh, pars[:l])))
           for l in range(3)]
    # measured: 14 plain; 8, 12, 12 with the best correction on 1x1, 2x2, 4x4 cells
    assert its[0] < its[1] <= its[2] < paper
    assert paper / its[1] < 1.4
