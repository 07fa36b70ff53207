"""Parity at the benchmark size (periodic 256 x 256 x 64 box, dx = 5 km, dz = 250 m) (GPU).

The oracle cannot factor this system, so it checks sampled outputs that it computes one by one
from its own cell matrices (rows of S x, of B_lambda and recovered cells), and properties that
hold at any size: the continuity defect of the recovered velocity equals the trace residual,
the preconditioner is a deterministic linear map, and the mixed-precision solve reaches the
same FP64 tolerance.  The launch configuration is the one the benchmark times.
"""

import numpy as np
import pytest

from gpu_common import dev, host, make_solver, rel_max, say
from oracle.hybrid import cell_recover, cell_rhs, cell_trace_operator
from oracle.local import local_matrices
from oracle.mesh import BoxMesh
from oracle.problem import cells_from_soa
from synth import make_box, make_rhs

NSAMPLE = 3000
_state = {}


def state():
    if not _state:
        say("[fullsize] building 256x256x64 problem")
        prob = make_box(nx=256, ny=256, nlev=64, dx=5e3, dz=250.0, dt=600.0, mg_levels=4)
        mesh = BoxMesh(prob.nx, prob.ny, prob.nlev, prob.dx, prob.dy, prob.z)
        fc, flf = mesh.face_cells()
        s = make_solver(prob)
        rng = np.random.default_rng(2024)
        faces = np.concatenate([rng.integers(0, mesh.n_zface, NSAMPLE // 2),
                                rng.integers(mesh.n_zface, mesh.ntrace, NSAMPLE // 2),
                                np.arange(mesh.ncol - 3, mesh.ncol + 3), [0, mesh.ntrace - 1]])
        cells = np.unique(np.concatenate([fc[faces][fc[faces] >= 0], rng.integers(0, mesh.ncell, NSAMPLE),
                                          [0, mesh.ncell - 1]]))
        loc = local_matrices(mesh, prob, cells=cells)
        _state.update(prob=prob, mesh=mesh, fc=fc, flf=flf, s=s, faces=faces, cells=cells, loc=loc,
                      pos={c: i for i, c in enumerate(cells)})
    return _state


def _rows(st, cellvals):
    """Sum over the (one or two) cells of each sampled face of cellvals[cell_index, local face]."""
    out = np.zeros(len(st["faces"]))
    for j, F in enumerate(st["faces"]):
        for side in range(2):
            c = st["fc"][F, side]
            if c >= 0:
                out[j] += cellvals(st["pos"][c], st["flf"][F, side])
    return out


@pytest.mark.gpu
def test_fullsize_trace_apply_rows():
    st = state()
    import torch

    mesh, s = st["mesh"], st["s"]
    x = np.random.default_rng(11).standard_normal(mesh.ntrace)
    y = torch.empty(mesh.ntrace, dtype=torch.float64, device="cuda")
    s.trace_apply(dev(x), y)
    Sc = cell_trace_operator(st["loc"])
    xc = x[mesh.cell_faces[st["cells"]]]  # (n, 6)
    ref = _rows(st, lambda i, a: Sc[i, a] @ xc[i])
    err = rel_max(host(y)[st["faces"]], ref)
    say(f"[fullsize trace_apply] sampled rows {len(ref)} rel err {err:.2e}")
    assert err <= 1e-12


@pytest.mark.gpu
def test_fullsize_condense_and_recover_samples():
    st = state()
    import torch

    prob, mesh, s, cells = st["prob"], st["mesh"], st["s"], st["cells"]
    r_ub, r_pi = make_rhs(prob, 0)
    ruc, rpc = cells_from_soa(r_ub, r_pi)
    b = torch.empty(mesh.ntrace, dtype=torch.float64, device="cuda")
    s.condense(dev(r_ub), dev(r_pi), b)
    bc = cell_rhs(st["loc"], ruc[cells], rpc[cells])
    ref = _rows(st, lambda i, a: bc[i, a])
    err_b = rel_max(host(b)[st["faces"]], ref)
    lam = np.random.default_rng(5).standard_normal(mesh.ntrace)
    ub = torch.empty(6 * mesh.ncell, dtype=torch.float64, device="cuda")
    pi = torch.empty(mesh.ncell, dtype=torch.float64, device="cuda")
    s.recover(dev(r_ub), dev(r_pi), dev(lam), ub, pi)
    u_ref, p_ref = cell_recover(st["loc"], lam[mesh.cell_faces[cells]], ruc[cells], rpc[cells])
    err_u = rel_max(host(ub).reshape(6, -1)[:, cells].T, u_ref)
    err_p = rel_max(host(pi)[cells], p_ref)
    say(f"[fullsize condense/recover] B {err_b:.2e} u {err_u:.2e} pi {err_p:.2e}")
    assert err_b <= 1e-12 and err_u <= 1e-12 and err_p <= 1e-12


@pytest.mark.gpu
def test_fullsize_preconditioner_is_a_deterministic_linear_map():
    st = state()
    import torch

    s, n = st["s"], st["mesh"].ntrace
    rng = np.random.default_rng(6)
    r1, r2 = dev(rng.standard_normal(n)), dev(rng.standard_normal(n))
    z1, z2, z3, z1b = (torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(4))
    s.precondition(r1, z1)
    s.precondition(r2, z2)
    s.precondition(2.0 * r1 - 3.0 * r2, z3)
    s.precondition(r1, z1b)
    assert torch.equal(z1, z1b)  # bitwise reproducible (no atomics)
    lin = float((z3 - (2.0 * z1 - 3.0 * z2)).abs().max() / z3.abs().max())
    say(f"[fullsize precondition] linearity defect {lin:.2e}")
    assert lin <= 1e-12


@pytest.mark.gpu
def test_fullsize_all_rows_residuals(tmp_path):
    """Solves at the benchmark size, FP64 to rtol 1e-12 and the mixed form to 1e-8, then recovery;
    the oracle builds every cell matrix (in chunks) and evaluates over all rows: ||B - S lambda|| /
    ||B||, the continuity defect of the recovered velocity (the sum of the two outward fluxes of
    every facet, = B - S lambda, Sec. 2.4) and the componentwise backward error of the recovered
    (u, Pi) in the unhybridised 2x2 system of Sec. 2.2, which must stay within what the continuity
    defect alone can cause (every cell satisfies its own equations at its recovered fluxes)."""
    import torch

    from gpu_common import oracle_all_rows

    st = state()
    prob, mesh = st["prob"], st["mesh"]
    r_ub, r_pi = make_rhs(prob, 1)
    sols, infos = [], []
    for precision, rtol in ((0, 1e-12), (1, 1e-8)):
        s = st["s"] if precision == 0 else make_solver(prob, precision=1)
        b = torch.empty(mesh.ntrace, dtype=torch.float64, device="cuda")
        lam = torch.zeros(mesh.ntrace, dtype=torch.float64, device="cuda")
        s.condense(dev(r_ub), dev(r_pi), b)
        info = s.solve(b, lam, rtol=rtol, maxit=500)
        ub = torch.empty(6 * mesh.ncell, dtype=torch.float64, device="cuda")
        pi = torch.empty(mesh.ncell, dtype=torch.float64, device="cuda")
        s.recover(dev(r_ub), dev(r_pi), lam, ub, pi)
        sols.append((host(lam), host(ub).reshape(6, -1).T.copy(), host(pi)))
        infos.append((precision, rtol, info))
        if precision:
            s.close()
    spec = dict(kind="box", nx=256, nlev=64, dx=5e3, dz=250.0, dt=600.0, mg_levels=4, seed=1)
    res = oracle_all_rows(spec, sols, tmp_path)
    for (precision, rtol, info), r in zip(infos, res):
        say(f"[fullsize all rows p{precision}] its {info['iters']} reported {info['rel_res']:.3e}, oracle "
            f"||B - S lambda||/||B|| {r['trace_res']:.3e}, continuity defect {r['defect_norm']:.3e} "
            f"(max entry {r['defect']:.1e}), 2x2 backward error {r['mixed_berr']:.1e} "
            f"(defect allows {r['mixed_berr_bound']:.1e})")
        assert info["status"] == 0 and info["rel_res"] <= rtol
        assert r["trace_res"] <= 1.05 * rtol
        assert abs(r["trace_res"] - info["rel_res"]) <= 0.05 * info["rel_res"]
        assert abs(r["defect_norm"] - r["trace_res"]) <= 0.05 * r["trace_res"]
        # the recovered (u, Pi) solves the 2x2 system up to its continuity defect: every row's
        # backward error within what |M| |x - X| of that defect allows (plus rounding)
        assert r["mixed_berr"] <= r["mixed_berr_bound"] + 1e-13
