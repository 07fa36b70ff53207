"""The paper's Configuration 1 on the GPU against the oracle: the unhybridised system of Sec. 2.2
(right-hand side and operator, to 1e-12 of the largest entry of each block), the approximate-Schur
preconditioner of Sec. 2.3 (1e-10), FGMRES on it (the oracle's residual estimates and iteration count; the
sparse LU solution), on a box, a ragged stretched box and a rotating cubed sphere; and the paper's ordering:
more iterations than the hybridised two-level method on the same problem."""

import numpy as np
import pytest

from gpu_common import dev, host, make_solver, say
from oracle.problem import OracleProblem, cells_from_soa
from oracle.schur import ApproximateSchur, MixedOperator, solve_configuration1
from synth import make_box, make_rhs, make_rhs_sphere, make_sphere

CASES = {
    "box16x16x8": (lambda: make_box(nx=16, ny=16, nlev=8, dx=10e3, dz=1250.0, mg_levels=4, perturb=0.05), make_rhs),
    "box9x7x13_stretched": (lambda: make_box(nx=9, ny=7, nlev=13, dx=5e3, dz=250.0, dt=600.0, mg_levels=1,
                                             perturb=0.1, stretch="quadratic", ztop=12e3, seed=3), make_rhs),
    "sphere_c8x10": (lambda: make_sphere(8, 10, mg_levels=3, perturb=0.05), make_rhs_sphere),
}


def _blocks_err(a, ref, nt):
    eu = np.abs(a[:nt] - ref[:nt]).max() / np.abs(ref[:nt]).max()
    ep = np.abs(a[nt:] - ref[nt:]).max() / np.abs(ref[nt:]).max()
    return eu, ep


@pytest.mark.gpu
@pytest.mark.parametrize("case", list(CASES))
def test_mixed_operator_and_preconditioner(case):
    import torch

    mk, rhs = CASES[case]
    prob = mk()
    s = make_solver(prob)
    o = OracleProblem(prob)
    op = MixedOperator(o.mixed)
    pc = ApproximateSchur(o.mixed, o.pc.mg.vcycle)
    nt, n = s.ntrace, s.nmixed
    assert n == op.n
    r_ub, r_pi = rhs(prob, 1)
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    s.mixed_rhs(dev(r_ub), dev(r_pi), b)
    bref = op.rhs(*cells_from_soa(r_ub, r_pi))
    eb = _blocks_err(host(b), bref, nt)
    x = op.expand(np.random.default_rng(7).standard_normal(o.mixed.nu + o.mixed.np_))
    y = torch.empty_like(b)
    s.mixed_apply(dev(x), y)
    ey = _blocks_err(host(y), op(x), nt)
    z = torch.empty_like(b)
    s.mixed_precondition(b, z)
    ez = _blocks_err(host(z), pc(bref), nt)
    say(f"[config 1] {case}: rhs {eb[0]:.1e}/{eb[1]:.1e}, A x {ey[0]:.1e}/{ey[1]:.1e}, "
        f"preconditioner {ez[0]:.1e}/{ez[1]:.1e}")
    assert max(eb) <= 1e-12 and max(ey) <= 1e-12 and max(ez) <= 1e-10
    assert np.all(host(y)[:nt][o.mesh.boundary] == 0.0) and np.all(host(z)[:nt][o.mesh.boundary] == 0.0)
    s.close()


@pytest.mark.gpu
# the tolerance stays above the rounding floor of the unweighted residual of this system (its rows
# differ in scale by 15 orders of magnitude; on the C8 sphere even the LU solution leaves ~2e-8).
# On the sphere the Hessenberg matrix of the restart cycle becomes numerically singular after
# 25-29 steps: from there on the oracle's own residual estimates stop decreasing monotonically
# (which a minimal-residual method cannot do in exact arithmetic; where this starts depends on the
# host's BLAS), and both sides' estimates, and with them the step at which they stop, are set by
# rounding (measured 48 against 51-54 iterations).  The residual histories are compared over the
# first 20 steps, the final count within 2 on the box and within a quarter on the sphere; the
# solutions against the sparse LU one to 1e-10 (measured 2.3e-11 on the box, 1.1e-11 on the sphere).
@pytest.mark.parametrize("case,rtol,band", [("box16x16x8", 1e-8, 2), ("sphere_c8x10", 1e-7, 0.25)])
def test_mixed_solve(case, rtol, band):
    import torch

    mk, rhs = CASES[case]
    prob = mk()
    s = make_solver(prob)
    o = OracleProblem(prob)
    op = MixedOperator(o.mixed)
    r_ub, r_pi = rhs(prob, 2)
    ruc, rpc = cells_from_soa(r_ub, r_pi)
    bref = op.rhs(ruc, rpc)
    _, hist, oits, conv = solve_configuration1(o.mixed, o.pc.mg.vcycle, bref, rtol=rtol)
    assert conv
    b = torch.empty(s.nmixed, dtype=torch.float64, device="cuda")
    s.mixed_rhs(dev(r_ub), dev(r_pi), b)
    x = torch.zeros_like(b)
    info = s.mixed_solve(b, x, rtol=rtol)
    xh = host(x)
    res = np.linalg.norm(bref - op(xh)) / np.linalg.norm(bref)
    u, pi = o.mixed.solve(ruc, rpc)
    ref = op.expand(np.concatenate([u, pi]))
    eu, ep = _blocks_err(xh, ref, s.ntrace)
    B = o.hyb.rhs(ruc, rpc)
    bl = dev(B)
    lam = torch.zeros_like(bl)
    its3c = s.solve(bl, lam, rtol=rtol)["iters"]
    say(f"[config 1] {case}: gpu {info['iters']} oracle {oits} iterations (3c: {its3c}), residual {res:.1e}, "
        f"error against LU {eu:.1e}/{ep:.1e}")
    assert info["status"] == 0 and res <= 1.05 * rtol
    np.testing.assert_allclose(info["history"][:20], hist[1:21], rtol=1e-3)  # measured 1.5e-4
    assert abs(info["iters"] - oits) <= (band if band >= 1 else max(2, int(band * oits)))
    assert eu <= 1e-10 and ep <= 1e-10
    assert info["iters"] > its3c
    s.close()
