"""Pins of the oracle's Configuration 1 (the approximate-Schur preconditioner on the unhybridised
system, Sec. 2.3), CPU only."""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.precond import lumped_velocity_mass, pressure_operator
from oracle.problem import OracleProblem, cells_from_soa
from oracle.schur import ApproximateSchur, MixedOperator, solve_configuration1
from synth import make_box, make_rhs, make_rhs_sphere, make_sphere


def _box():
    return make_box(nx=8, ny=6, nlev=6, dx=10e3, dz=1250.0, mg_levels=2, perturb=0.05)


def test_layout_round_trip_and_operator():
    """The library layout holds zeros on the ground / lid facets and the operator is the assembled
    mixed matrix on the interior dofs."""
    o = OracleProblem(_box(), with_precond=False)
    op = MixedOperator(o.mixed)
    rng = np.random.default_rng(1)
    x = op.expand(rng.standard_normal(o.mixed.nu + o.mixed.np_))
    assert np.all(x[: op.nt][o.mesh.boundary] == 0.0)
    np.testing.assert_array_equal(op.expand(op.compress(x)), x)
    y = op(x)
    assert np.all(y[: op.nt][o.mesh.boundary] == 0.0)
    np.testing.assert_allclose(op.compress(y), o.mixed.matrix @ op.compress(x), rtol=1e-14, atol=0)


def test_steps_invert_the_lumped_system():
    """With an exact solve of H in Step 2, Steps 1-3 are the exact inverse of the block system whose
    velocity block is the lumped mass (box and rotating sphere): any dropped term, wrong sign or
    transposed coupling breaks this identity."""
    for prob in (_box(), make_sphere(4, 4, mg_levels=2, perturb=0.05)):
        o = OracleProblem(prob, with_precond=False)
        m = o.mixed
        H = pressure_operator(m).tocsc()
        lu = spla.splu(H)
        pc = ApproximateSchur(m, lu.solve)
        A_l = sp.bmat([[sp.diags(lumped_velocity_mass(m)), m.G], [m.Bp, m.M3pi]], format="csr")
        x = np.random.default_rng(2).standard_normal(m.nu + m.np_)
        r = A_l @ x
        y = pc.op.compress(pc(pc.op.expand(r)))
        # the pressure exactly; the velocity, which Step 3 obtains from the cancellation of R_u and
        # G Pi (rows of this system differ by 15 orders of magnitude; even a dense LU solve leaves
        # 1e-3 there), by the componentwise backward error of the whole block system
        np.testing.assert_allclose(y[m.nu :], x[m.nu :], rtol=0, atol=1e-11 * np.abs(x[m.nu :]).max())
        berr = np.abs(r - A_l @ y) / (abs(A_l) @ np.abs(y) + np.abs(r))
        assert berr.max() <= 1e-9
        # a dropped term is caught: Step 3 without G Pi, Step 1 without the velocity part
        y_bad = y.copy()
        y_bad[: m.nu] = r[: m.nu] / lumped_velocity_mass(m)
        assert (np.abs(r - A_l @ y_bad) / (abs(A_l) @ np.abs(y_bad) + np.abs(r))).max() > 1e-3
        p_bad = lu.solve(r[m.nu :])
        assert np.abs(p_bad - x[m.nu :]).max() > 1e-3 * np.abs(x[m.nu :]).max()


def test_configuration1_solves_the_mixed_system():
    """FGMRES with the approximate-Schur preconditioner (one V-cycle in Step 2) reaches the
    tolerance and the sparse LU solution of the mixed system, which is also the hybridised solution
    (box and sphere); it needs more iterations than the hybridised two-level method (the paper's
    ordering of Configurations 1 and 3c)."""
    for prob, rhs in ((make_box(nx=12, ny=12, nlev=8, dx=10e3, dz=1250.0, mg_levels=3, perturb=0.05),
                       make_rhs),
                      (make_sphere(8, 10, mg_levels=3, perturb=0.05), make_rhs_sphere)):
        o = OracleProblem(prob)
        ruc, rpc = cells_from_soa(*rhs(prob, 1))
        op = MixedOperator(o.mixed)
        b = op.rhs(ruc, rpc)
        # 1e-8, the benchmark's tolerance: the rows of this system differ in scale by 15 orders of
        # magnitude, and the residual of even the LU solution is 1e-10 of b in the pressure rows
        x, hist, its, conv = solve_configuration1(o.mixed, o.pc.mg.vcycle, b, rtol=1e-8)
        assert conv and hist[-1] <= 1e-8
        assert np.linalg.norm(b - op(x)) <= 1.01e-8 * np.linalg.norm(b)
        u, pi = o.mixed.solve(ruc, rpc)
        ref = op.expand(np.concatenate([u, pi]))
        assert np.abs(x[op.nt :] - ref[op.nt :]).max() <= 1e-6 * np.abs(ref[op.nt :]).max()
        assert np.abs(x[: op.nt] - ref[: op.nt]).max() <= 1e-6 * np.abs(ref[: op.nt]).max()
        B = o.hyb.rhs(ruc, rpc)
        its3c = o.solve_fgmres(B, rtol=1e-8)[2]
        assert its > its3c
