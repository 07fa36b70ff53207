"""Order 1 (RT1 / DG1 / Q1 trace) on the GPU against the p = 1 oracle: the trace operator, the
condensed right-hand side and the recovery on small boxes (element by element), and sampled rows
and cells on the 128x128x32 box (dx = 10 km, dz = 500 m) in the launch configuration of the
benchmark."""

import numpy as np
import pytest

from gpu_common import dev, host, params_for, rel_max, say
from oracle import p1 as op1
from oracle.mesh import BoxMesh
from paper_2210_11797_amd import HybSolver, levels_of
from synth import make_box, make_rhs_p1

CASES = {
    "3x2x3": dict(nx=3, ny=2, nlev=3, dx=5e3, dz=250.0, perturb=0.05),
    "8x6x5": dict(nx=8, ny=6, nlev=5, dx=5e3, dz=250.0, perturb=0.1, theta_col_perturb=0.02),
    "stretched": dict(nx=4, ny=4, nlev=9, dx=10e3, dz=None, stretch="quadratic", ztop=16e3),
    # an odd number of columns: S x one cell per thread (two cells per thread where ncol is even)
    "odd_3x3x4": dict(nx=3, ny=3, nlev=4, dx=5e3, dz=250.0, perturb=0.05),
}


def make_p1_solver(prob, **kw):
    s = HybSolver(prob.nlev, levels_of(prob), prob.dx, prob.dy, prob.dz, params_for(prob, **kw), order=1)
    s.assemble_local(dev(prob.theta_w), dev(prob.exner_hat_w), dev(prob.exner_c), dev(prob.rho_c))
    s.condense()
    return s


def _box(kw):
    kw = dict(kw)
    if kw.get("dz") is None:
        kw.pop("dz")
    return make_box(mg_levels=1, **kw)


@pytest.mark.gpu
@pytest.mark.parametrize("case", list(CASES))
def test_p1_operators_match_oracle(case):
    prob = _box(CASES[case])
    say(f"[p1] case {case}: {prob.nx}x{prob.ny}x{prob.nlev}")
    s = make_p1_solver(prob)
    mesh = BoxMesh(prob.nx, prob.ny, prob.nlev, prob.dx, prob.dy, prob.z)
    h = op1.HybridP1(mesh, op1.local_matrices(mesh, prob))
    assert s.ntrace == h.ntrace
    import torch

    rng = np.random.default_rng(1)
    x = rng.standard_normal(s.ntrace)
    y = torch.empty(s.ntrace, dtype=torch.float64, device="cuda")
    s.trace_apply(dev(x), y)
    e_s = rel_max(host(y), h.S @ x)
    r_u, r_p = make_rhs_p1(prob, 2)
    b = torch.empty_like(y)
    s.condense(dev(r_u), dev(r_p), b)
    ruc, rpc = r_u.reshape(36, -1).T.copy(), r_p.reshape(8, -1).T.copy()
    e_b = rel_max(host(b), h.rhs(ruc, rpc))
    u = torch.empty(36 * s.ncell, dtype=torch.float64, device="cuda")
    pi = torch.empty(8 * s.ncell, dtype=torch.float64, device="cuda")
    s.recover(dev(r_u), dev(r_p), dev(x), u, pi)
    uref, pref = h.recover(x, ruc, rpc)
    e_u = rel_max(host(u).reshape(36, -1).T, uref)
    e_p = rel_max(host(pi).reshape(8, -1).T, pref)
    say(f"[p1] {case}: S x {e_s:.1e}, B {e_b:.1e}, u {e_u:.1e}, pi {e_p:.1e}")
    assert max(e_s, e_b) <= 1e-11 and max(e_u, e_p) <= 1e-10


@pytest.mark.gpu
def test_p1_fullsize_sampled_rows():
    """128x128x32: 2000 sampled rows of S x and 500 sampled cells of the recovery against the oracle's
    own cell matrices for the cells involved."""
    import torch

    prob = make_box(nx=128, ny=128, nlev=32, dx=10e3, dz=500.0, mg_levels=1)
    s = make_p1_solver(prob)
    mesh = BoxMesh(prob.nx, prob.ny, prob.nlev, prob.dx, prob.dy, prob.z)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(s.ntrace)
    y = torch.empty(s.ntrace, dtype=torch.float64, device="cuda")
    s.trace_apply(dev(x), y)
    yh = host(y)
    rows = rng.choice(s.ntrace, 2000, replace=False)
    facets = rows // 4
    # the (cell, local face) pairs of each sampled facet
    owner = {}
    sel = np.isin(mesh.cell_faces, facets)
    for c_, f_ in zip(*np.nonzero(sel)):
        owner.setdefault(int(mesh.cell_faces[c_, f_]), []).append((int(c_), int(f_)))
    need = sorted({c_ for v in owner.values() for c_, _ in v})
    loc = op1.local_matrices(mesh, prob, cells=np.array(need))
    SK = dict(zip(need, op1.cell_trace_operator(loc)))
    dofs = op1.cell_dofs(mesh)
    ref = np.zeros(len(rows))
    for n_, T in enumerate(rows):
        for c_, f_ in owner[int(T // 4)]:
            ref[n_] += SK[c_][4 * f_ + T % 4] @ x[dofs[c_]]
    e_s = np.abs(yh[rows] - ref).max() / np.abs(ref).max()
    r_u, r_p = make_rhs_p1(prob, 4)
    u = torch.empty(36 * s.ncell, dtype=torch.float64, device="cuda")
    pi = torch.empty(8 * s.ncell, dtype=torch.float64, device="cuda")
    s.recover(dev(r_u), dev(r_p), dev(x), u, pi)
    cs = rng.choice(s.ncell, 500, replace=False)
    locc = op1.local_matrices(mesh, prob, cells=cs)
    ruc, rpc = r_u.reshape(36, -1).T[cs], r_p.reshape(8, -1).T[cs]
    R = np.concatenate([ruc, rpc], axis=1)
    R[:, :36] -= np.einsum("caf,cf->ca", locc["K"], x[dofs[cs]])
    X = np.linalg.solve(locc["A"], R[:, :, None])[:, :, 0]
    uh = host(u).reshape(36, -1).T[cs]
    ph = host(pi).reshape(8, -1).T[cs]
    e_u = np.abs(uh - X[:, :36]).max() / np.abs(X[:, :36]).max()
    e_p = np.abs(ph - X[:, 36:]).max() / np.abs(X[:, 36:]).max()
    say(f"[p1] 128x128x32 sampled: S x {e_s:.1e}, u {e_u:.1e}, pi {e_p:.1e}")
    assert e_s <= 1e-11 and max(e_u, e_p) <= 1e-10


@pytest.mark.gpu
@pytest.mark.parametrize("size", ["8x6x5", "odd_3x3x4", "128x128x32"])
def test_p1_mfma_condensation_error_vs_fp64(size):
    """S_K condensed on matrix cores against the FP64 condensation: FP32 MFMA to 1e-5 and BF16 split
    hi + lo (three products, FP32 accumulation) to 1e-4 of the largest entry of S x; the elimination
    without pivoting in FP32 loses about cond(A_K) * 2^-24 on A_K, far less on the condensed block
    (~1e-6 measured)."""
    import torch

    from paper_2210_11797_amd import PREC_FP64, PREC_MFMA_BF16X, PREC_MFMA_FP32

    if size in CASES:
        prob = _box(CASES[size])
    else:
        prob = make_box(nx=128, ny=128, nlev=32, dx=10e3, dz=500.0, mg_levels=1)
    rng = np.random.default_rng(8)
    x = dev(rng.standard_normal(4 * (prob.ncol * (prob.nlev + 1) + 2 * prob.ncol * prob.nlev)))
    out = {}
    for prec in (PREC_FP64, PREC_MFMA_FP32, PREC_MFMA_BF16X):
        s = HybSolver(prob.nlev, levels_of(prob), prob.dx, prob.dy, prob.dz, params_for(prob, precision=prec), order=1)
        s.assemble_local(dev(prob.theta_w), dev(prob.exner_hat_w), dev(prob.exner_c), dev(prob.rho_c))
        s.condense()
        y = torch.empty(s.ntrace, dtype=torch.float64, device="cuda")
        s.trace_apply(x, y)
        out[prec] = host(y)
        s.close()
        del s
        torch.cuda.empty_cache()
    e32 = rel_max(out[PREC_MFMA_FP32], out[PREC_FP64])
    ebf = rel_max(out[PREC_MFMA_BF16X], out[PREC_FP64])
    say(f"[p1] {size}: S x error vs FP64 condensation: FP32 MFMA {e32:.1e}, BF16 split MFMA {ebf:.1e}")
    assert e32 <= 1e-5 and ebf <= 1e-4


PRECOND_CASES = {
    "4x4x4": dict(nx=4, ny=4, nlev=4, dx=5e3, dz=250.0, perturb=0.05, mg_levels=2),
    "8x6x5": dict(nx=8, ny=6, nlev=5, dx=5e3, dz=250.0, perturb=0.1, mg_levels=2),
    "stretched": dict(nx=8, ny=8, nlev=9, dx=10e3, ztop=16e3, stretch="quadratic", mg_levels=3),
}


@pytest.mark.gpu
@pytest.mark.parametrize("case", list(PRECOND_CASES))
def test_p1_precondition_and_solve_match_oracle(case):
    """The order-1 two-level preconditioner against the oracle's (a fixed linear map of ~50 column
    solves and a V-cycle: compared to 1e-9), and FGMRES to rtol 1e-12 against the direct solution
    (1e-9), with the oracle's FGMRES iteration count (+-1)."""
    import torch
    import scipy.sparse.linalg as spla

    from oracle.krylov import fgmres
    from oracle.problem import OracleProblem

    prob = make_box(**PRECOND_CASES[case])
    say(f"[p1] precondition/solve case {case}")
    s = make_p1_solver(prob)
    mesh = BoxMesh(prob.nx, prob.ny, prob.nlev, prob.dx, prob.dy, prob.z)
    h = op1.HybridP1(mesh, op1.local_matrices(mesh, prob))
    tl = op1.TwoLevelP1(mesh, h.S, OracleProblem(prob).H, mg_levels=len(prob.levels))
    r_u, r_p = make_rhs_p1(prob, 5)
    B = h.rhs(r_u.reshape(36, -1).T.copy(), r_p.reshape(8, -1).T.copy())
    z = torch.empty(s.ntrace, dtype=torch.float64, device="cuda")
    s.precondition(dev(B), z)
    zref = tl(B)
    e_m = rel_max(host(z), zref)
    b = torch.empty_like(z)
    s.condense(dev(r_u), dev(r_p), b)
    lam = torch.zeros_like(z)
    info = s.solve(b, lam, rtol=1e-12, maxit=500)
    lref = spla.splu(h.S.tocsc()).solve(B)
    e_l = rel_max(host(lam), lref)
    its_ref = fgmres(lambda v: h.S @ v, tl, B, rtol=1e-12, restart=30, maxit=500)[2]
    say(f"[p1] {case}: M(B) {e_m:.1e}; solve {info['iters']} its (oracle {its_ref}), lambda {e_l:.1e}")
    assert e_m <= 1e-9
    assert info["status"] == 0 and e_l <= 1e-9 and abs(info["iters"] - its_ref) <= 1


@pytest.mark.gpu
def test_p1_mixed_form_reaches_fp64_tolerance():
    """The mixed form at order 1 (S_K condensed in FP64 for the outer operator, its FP32 copy in the
    preconditioner): the preconditioner differs from the FP64 one by FP32 rounding, FGMRES reaches
    the FP64 tolerance on the FP64 operator (measured by the oracle), and the solution agrees with
    the direct solution as that tolerance allows."""
    import torch
    import scipy.sparse.linalg as spla

    from paper_2210_11797_amd import PREC_MIXED

    prob = make_box(**PRECOND_CASES["8x6x5"])
    say("[p1] mixed form 8x6x5")
    s64 = make_p1_solver(prob)
    smx = make_p1_solver(prob, precision=PREC_MIXED)
    mesh = BoxMesh(prob.nx, prob.ny, prob.nlev, prob.dx, prob.dy, prob.z)
    h = op1.HybridP1(mesh, op1.local_matrices(mesh, prob))
    r_u, r_p = make_rhs_p1(prob, 6)
    B = h.rhs(r_u.reshape(36, -1).T.copy(), r_p.reshape(8, -1).T.copy())
    z64, zmx = (torch.empty(s64.ntrace, dtype=torch.float64, device="cuda") for _ in range(2))
    s64.precondition(dev(B), z64)
    smx.precondition(dev(B), zmx)
    e_z = rel_max(host(zmx), host(z64))
    b = torch.empty_like(z64)
    smx.condense(dev(r_u), dev(r_p), b)
    lam = torch.zeros_like(z64)
    info = smx.solve(b, lam, rtol=1e-8, maxit=500)
    res = np.linalg.norm(B - h.S @ host(lam)) / np.linalg.norm(B)
    lref = spla.splu(h.S.tocsc()).solve(B)
    e_l = np.linalg.norm(host(lam) - lref) / np.linalg.norm(lref)
    say(f"[p1 mixed] M(B) vs FP64 {e_z:.1e}; {info['iters']} its, oracle residual {res:.1e}, lambda {e_l:.1e}")
    assert 0 < e_z <= 1e-5
    assert info["status"] == 0 and res <= 1e-8 and e_l <= 1e-5
