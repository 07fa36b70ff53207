"""Pins of the oracle's cell matrices (CPU only).

The oracle integrates the bilinear forms numerically on the basis functions;
here they are compared with closed forms worked out by hand for an
axis-aligned cell (exact integrals of products of linear functions, the
divergence theorem for g and k, the one-point rule for the pressure row).
"""

import numpy as np
import pytest

from oracle.local import local_matrices
from oracle.mesh import BoxMesh
from synth import make_box


def _closed_form(prob, mesh):
    n = mesh.ncell
    k = mesh.cell_layer
    col = mesh.cell_iy * mesh.nx + mesh.cell_ix
    hx, hy, hz = mesh.dx, mesh.dy, mesh.dz[k]
    vol = hx * hy * hz
    thB, thT = prob.theta_w[k, col], prob.theta_w[k + 1, col]
    piB, piT = prob.exner_hat_w[k, col], prob.exner_hat_w[k + 1, col]
    dt, tu, tr, tt, cp, kap = prob.dt, prob.tau_u, prob.tau_rho, prob.tau_theta, prob.cp, prob.kappa
    ax, ay, az = hx / (hy * hz), hy / (hx * hz), hz / (hx * hy)
    beta = -tu * tt * dt**2 * cp * (piT - piB) * (thT - thB) / hz**2
    m = np.array([[1 / 3, -1 / 6], [-1 / 6, 1 / 3]])
    A = np.zeros((n, 7, 7))
    A[:, 0:2, 0:2] = ax[..., None, None] * m if np.ndim(ax) else ax * m
    A[:, 2:4, 2:4] = ay[..., None, None] * m if np.ndim(ay) else ay * m
    A[:, 4:6, 4:6] = ((1 + beta) * az)[:, None, None] * m
    thbar = np.stack([0.5 * (thB + thT)] * 4 + [thB, thT], axis=1)
    g = -tu * dt * cp * thbar
    A[:, :6, 6] = g
    q = tt * dt * (thT - thB) / (thT + thB)
    d = np.full((n, 6), tr * dt)
    d[:, 4] -= q
    d[:, 5] += q
    A[:, 6, :6] = d
    A[:, 6, 6] = (1 - kap) / kap * vol / prob.exner_c[k, col]
    K = np.zeros((n, 6, 6))
    K[:, np.arange(6), np.arange(6)] = -g
    return A, K


@pytest.mark.parametrize(
    "kw",
    [
        dict(nx=3, ny=4, nlev=5, dx=10e3, dy=7e3, dz=800.0, mg_levels=1, perturb=0.1),
        dict(nx=4, ny=3, nlev=6, dx=5e3, dy=5e3, ztop=30e3, stretch="quadratic", mg_levels=1, theta_col_perturb=0.05),
        dict(nx=2, ny=2, nlev=3, dx=1e3, dy=2e3, dz=50.0, mg_levels=1, nbv=0.0),
    ],
)
def test_cell_matrices_match_closed_form(kw):
    prob = make_box(**kw)
    mesh = BoxMesh(prob.nx, prob.ny, prob.nlev, prob.dx, prob.dy, prob.z)
    loc = local_matrices(mesh, prob)
    A, K = _closed_form(prob, mesh)
    scale = np.abs(A).max(axis=(1, 2), keepdims=True)
    # row/column scales differ by orders of magnitude: compare blockwise
    for rs, cs in ((slice(0, 6), slice(0, 6)), (slice(0, 6), slice(6, 7)), (slice(6, 7), slice(0, 6)), (slice(6, 7), slice(6, 7))):
        ref = A[:, rs, cs]
        err = np.abs(loc["A"][:, rs, cs] - ref).max()
        assert err <= 1e-13 * np.abs(ref).max(), (rs, cs, err)
    assert np.abs(loc["K"] - K).max() <= 1e-13 * np.abs(K).max()
    # c(v_a, nu_f) = delta_af: each basis function has unit flux through its own face only
    assert np.abs(loc["C"] - np.eye(6)).max() <= 1e-14
    assert scale.min() > 0


def test_divergence_and_lagrange_identity():
    """Each basis function has divergence integral 1; A (0,..,0,-1)^T = (k; -m_K) (k = -g)."""
    prob = make_box(nx=3, ny=3, nlev=4, dx=9e3, dy=6e3, dz=500.0, mg_levels=1, perturb=0.2)
    mesh = BoxMesh(prob.nx, prob.ny, prob.nlev, prob.dx, prob.dy, prob.z)
    loc = local_matrices(mesh, prob)
    # D_{K,F} = tau_rho dt rho* int div v_F  ->  int div v_F = 1
    q = loc["q32"]
    draw = (loc["d"] - q) * loc["m3"][:, None] / loc["m3rho"][:, None]
    rho = prob.rho_c.reshape(-1)
    np.testing.assert_allclose(draw / (prob.tau_rho * prob.dt * rho[:, None]), 1.0, rtol=1e-13)
    e = np.zeros(7)
    e[6] = -1.0
    lhs = loc["A"] @ e
    kdiag = loc["K"][:, np.arange(6), np.arange(6)]
    np.testing.assert_allclose(lhs[:, :6], kdiag, rtol=1e-13)
    np.testing.assert_allclose(lhs[:, 6], -loc["A"][:, 6, 6], rtol=1e-15)


def test_local_sizes_match_table_of_unknowns(golden_dir):
    rows = [list(map(int, ln.split())) for ln in open(f"{golden_dir}/table5_dofs.txt") if ln.strip() and not ln.startswith("#")]
    p0 = rows[0]
    assert p0[0] == 0
    prob = make_box(nx=3, ny=3, nlev=3, dx=1e4, dz=1e3, mg_levels=1)
    mesh = BoxMesh(prob.nx, prob.ny, prob.nlev, prob.dx, prob.dy, prob.z)
    loc = local_matrices(mesh, prob)
    n_p = 1  # one W3 dof per cell
    n_u_local = loc["A"].shape[1] - n_p  # broken velocity dofs of a cell
    n_lam_local = loc["K"].shape[2]  # trace dofs touching a cell
    # facet unknowns are shared by two cells -> weight 1/2
    assert (p0[1], p0[2], p0[3], p0[4]) == (n_p, n_u_local // 2, n_p + n_u_local // 2, n_lam_local // 2)
    assert p0[5] == loc["A"].shape[1] == 7
    assert p0[6] == loc["K"].shape[1] == 6
    # a periodic column of L cells has 3L+1 trace facets per column -> 3 per cell as L grows
    assert mesh.ntrace == mesh.ncol * (3 * mesh.nlev + 1)
