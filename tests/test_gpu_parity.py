"""Parity of every C-ABI call against the CPU FP64 oracle (GPU).

Sizes: several column tiles (64 columns per wavefront) with ragged tails, a stretched grid,
a horizontally varying theta* (hybrid operator only), and degenerate 2x2x1 meshes.
Tolerances (FP64): operator application, condensation and recovery 1e-12 relative to the
largest entry; the preconditioner (a fixed linear map) 100 eps cond(H); a solve to rtol 1e-15
against the sparse direct solutions and against the oracle's FGMRES iterate after the same number
of steps 1e-10 (relative 2-norm).
"""

import numpy as np
import pytest

from gpu_common import dev, host, make_solver, rel_max, rel_norm, say
from oracle.problem import OracleProblem, cells_from_soa
from synth import make_box, make_rhs

CASES = {
    "box16": dict(nx=16, ny=16, nlev=8, dx=10e3, dz=1250.0, mg_levels=4, perturb=0.05),
    "ragged": dict(nx=12, ny=10, nlev=5, dx=7e3, dy=5e3, dz=400.0, mg_levels=2, perturb=0.1),
    "tiles": dict(nx=24, ny=20, nlev=6, dx=5e3, dz=500.0, mg_levels=3, perturb=0.02),
    "aniso": dict(nx=16, ny=16, nlev=16, dx=5e3, dz=250.0, mg_levels=4, perturb=0.02),
    "stretched": dict(nx=8, ny=8, nlev=30, dx=48e3, ztop=30e3, stretch="quadratic", dt=1800.0, mg_levels=3),
    "theta_varies": dict(nx=10, ny=6, nlev=4, dx=10e3, dz=1000.0, mg_levels=2, theta_col_perturb=0.03),
    "tiny": dict(nx=2, ny=2, nlev=1, dx=10e3, dz=1000.0, mg_levels=1),
}

_cache = {}


def setup(name):
    if name not in _cache:
        say(f"[setup] case {name}: {CASES[name]}")
        prob = make_box(**CASES[name])
        orc = OracleProblem(prob, with_mixed=True, with_precond=True)
        s = make_solver(prob)
        _cache[name] = (prob, orc, s)
    return _cache[name]


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(CASES))
def test_trace_apply(name):
    prob, orc, s = setup(name)
    import torch

    rng = np.random.default_rng(1)
    x = rng.standard_normal(orc.mesh.ntrace)
    y = torch.empty(orc.mesh.ntrace, dtype=torch.float64, device="cuda")
    s.trace_apply(dev(x), y)
    ref = orc.hyb.S @ x
    err = rel_max(host(y), ref)
    say(f"[trace_apply] {name}: rel err {err:.2e}")
    assert err <= 1e-12


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(CASES))
def test_condense_rhs_and_recover(name):
    prob, orc, s = setup(name)
    import torch

    r_ub, r_pi = make_rhs(prob, 7)
    ruc, rpc = cells_from_soa(r_ub, r_pi)
    b = torch.empty(orc.mesh.ntrace, dtype=torch.float64, device="cuda")
    s.condense(dev(r_ub), dev(r_pi), b)
    Bref = orc.hyb.rhs(ruc, rpc)
    err_b = rel_max(host(b), Bref)
    lam, ub_ref, pi_ref, _ = orc.hyb.solve_direct(ruc, rpc)
    ub = torch.empty(6 * orc.mesh.ncell, dtype=torch.float64, device="cuda")
    pi = torch.empty(orc.mesh.ncell, dtype=torch.float64, device="cuda")
    s.recover(dev(r_ub), dev(r_pi), dev(lam), ub, pi)
    err_u = rel_max(host(ub).reshape(6, -1).T, ub_ref)
    err_p = rel_max(host(pi), pi_ref)
    say(f"[condense/recover] {name}: B {err_b:.2e} u {err_u:.2e} pi {err_p:.2e}")
    assert err_b <= 1e-12 and err_u <= 1e-12 and err_p <= 1e-12


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(CASES))
def test_precondition(name):
    prob, orc, s = setup(name)
    import torch

    rng = np.random.default_rng(3)
    r = rng.standard_normal(orc.mesh.ntrace)
    z = torch.empty(orc.mesh.ntrace, dtype=torch.float64, device="cuda")
    s.precondition(dev(r), z)
    ref = orc.pc(r)
    err = rel_max(host(z), ref)
    # both sides apply the same fixed linear map with backward-stable column solves in different
    # rounding orders; the map contains the coarsest-level sweeps (an approximate H^-1), so the
    # difference is bounded by a modest multiple of cond(H) * eps
    cond_h = np.linalg.cond(orc.H.toarray())
    tol = max(1e-12, 100 * np.finfo(float).eps * cond_h)
    say(f"[precondition] {name}: rel err {err:.2e} (cond(H) {cond_h:.1e}, tol {tol:.1e})")
    assert err <= tol


COARSEST = {
    # damped block-Jacobi sweeps on the coarsest level instead of the Chebyshev semi-iteration
    "jacobi30": (dict(nx=24, ny=20, nlev=6, dx=5e3, dz=500.0, mg_levels=3, perturb=0.02),
                 dict(mg_coarse_sweeps=30, mg_coarse_cheb=None), dict(mg_coarse_sweeps=30, mg_coarse_cheb=0)),
    # more than 64 levels: the coarsest Chebyshev steps take the residual + column-solve kernels
    "cheb_nlev70": (dict(nx=8, ny=8, nlev=70, dx=5e3, dz=150.0, mg_levels=2, perturb=0.02), {}, {}),
    # a longer Chebyshev solve on another interval
    "cheb12": (dict(nx=16, ny=16, nlev=8, dx=10e3, dz=1250.0, mg_levels=4, perturb=0.05),
               dict(mg_coarse_sweeps=12, mg_coarse_cheb=(0.05, 1.9)),
               dict(mg_coarse_sweeps=12, cheb_lo=0.05, cheb_hi=1.9)),
}


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(COARSEST))
def test_precondition_coarsest_variants(name):
    import torch

    box, okw, gkw = COARSEST[name]
    say(f"[setup] coarsest variant {name}: {box} oracle {okw} library {gkw}")
    prob = make_box(**box)
    orc = OracleProblem(prob, with_mixed=True, with_precond=True, **okw)
    s = make_solver(prob, **gkw)
    rng = np.random.default_rng(4)
    r = rng.standard_normal(orc.mesh.ntrace)
    z = torch.empty(orc.mesh.ntrace, dtype=torch.float64, device="cuda")
    s.precondition(dev(r), z)
    ref = orc.pc(r)
    err = rel_max(host(z), ref)
    cond_h = np.linalg.cond(orc.H.toarray())
    tol = max(1e-12, 100 * np.finfo(float).eps * cond_h)
    say(f"[precondition] {name}: rel err {err:.2e} (cond(H) {cond_h:.1e}, tol {tol:.1e})")
    assert err <= tol
    lam = torch.zeros(orc.mesh.ntrace, dtype=torch.float64, device="cuda")
    b = dev(rng.standard_normal(orc.mesh.ntrace))
    info = s.solve(b, lam, rtol=1e-10, maxit=300)
    assert info["status"] == 0
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["box16", "ragged", "tiles", "stretched", "tiny", "aniso"])
def test_solve_matches_direct(name):
    """FP64 solve to rtol 1e-15 (the rounding floor of the trace residual) against the oracle's
    sparse direct solutions: lambda, and (u, Pi) after the recovery against the mixed system, to
    1e-10 relative; and against the oracle's own FGMRES iterate after the same number of steps
    (the same Krylov space and preconditioner) to 1e-10."""
    prob, orc, s = setup(name)
    import torch

    from oracle.krylov import fgmres

    r_ub, r_pi = make_rhs(prob, 0)
    ruc, rpc = cells_from_soa(r_ub, r_pi)
    lam_ref, ub_ref, pi_ref, Bref = orc.hyb.solve_direct(ruc, rpc)
    u_mixed, pi_mixed = orc.mixed.solve(ruc, rpc)
    b = torch.empty(orc.mesh.ntrace, dtype=torch.float64, device="cuda")
    lam = torch.zeros(orc.mesh.ntrace, dtype=torch.float64, device="cuda")
    s.condense(dev(r_ub), dev(r_pi), b)
    info = s.solve(b, lam, rtol=1e-15, maxit=300)
    ub = torch.empty(6 * orc.mesh.ncell, dtype=torch.float64, device="cuda")
    pi = torch.empty(orc.mesh.ncell, dtype=torch.float64, device="cuda")
    s.recover(dev(r_ub), dev(r_pi), lam, ub, pi)
    e_l = rel_norm(host(lam), lam_ref)
    e_p = rel_norm(host(pi), pi_mixed)
    e_u = rel_norm(host(ub).reshape(6, -1).T, orc.mixed.broken_from_continuous(u_mixed))
    # residual and backward error measured by the oracle with its own operators
    res = np.linalg.norm(Bref - orc.hyb.S @ host(lam)) / np.linalg.norm(Bref)
    ubh = host(ub).reshape(6, -1).T
    uc = np.zeros(orc.mixed.nu)
    for a in range(6):
        dd = orc.mixed.udof[orc.mesh.cell_faces[:, a]]
        ok = dd >= 0
        uc[dd[ok]] = orc.mesh.cell_sign[ok, a] * ubh[ok, a]
    berr = orc.mixed.backward_error(uc, host(pi), ruc, rpc)
    # the oracle's FGMRES (restart 30, the two-level preconditioner) run for the same number of steps
    x_it, _, its_o, _ = fgmres(lambda v: orc.hyb.S @ v, orc.pc, Bref, rtol=0.0, restart=30, maxit=info["iters"])
    e_it = rel_norm(host(lam), x_it)
    say(f"[solve] {name}: its {info['iters']} res {info['rel_res']:.2e} oracle res {res:.2e} backward err "
        f"{berr:.2e} lam {e_l:.2e} pi {e_p:.2e} u {e_u:.2e}; vs the oracle's iterate after {its_o} steps {e_it:.2e}")
    assert info["status"] == 0 and info["rel_res"] <= 1e-15 and res <= 2e-15
    assert its_o == info["iters"] and e_it <= 1e-10
    assert e_l <= 1e-10 and e_p <= 1e-10 and e_u <= 1e-10
    assert berr <= 1e-10


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["box16", "tiles"])
def test_iterations_match_oracle(name):
    """With a fixed linear preconditioner, the FGMRES histories of oracle and GPU agree."""
    prob, orc, s = setup(name)
    import torch

    r_ub, r_pi = make_rhs(prob, 4)
    ruc, rpc = cells_from_soa(r_ub, r_pi)
    Bref = orc.hyb.rhs(ruc, rpc)
    _, hist, its, conv = orc.solve_fgmres(Bref, rtol=1e-8)
    b = dev(Bref)
    lam = torch.zeros_like(b)
    info = s.solve(b, lam, rtol=1e-8, maxit=200)
    say(f"[iterations] {name}: gpu {info['iters']} oracle {its}")
    assert abs(info["iters"] - its) <= 1
    n = min(len(info["history"]), len(hist) - 1)
    np.testing.assert_allclose(info["history"][:n], hist[1 : n + 1], rtol=1e-6)


@pytest.mark.gpu
def test_mixed_precision_reaches_fp64_tolerance():
    prob, orc, s = setup("tiles")
    import torch

    from gpu_common import make_solver as mk

    sm = mk(prob, precision=1)
    r_ub, r_pi = make_rhs(prob, 5)
    ruc, rpc = cells_from_soa(r_ub, r_pi)
    lam_ref, _, _, Bref = orc.hyb.solve_direct(ruc, rpc)
    b = dev(Bref)
    lam = torch.zeros_like(b)
    info = sm.solve(b, lam, rtol=1e-8, maxit=200)
    true_res = np.linalg.norm(Bref - orc.hyb.S @ host(lam)) / np.linalg.norm(Bref)
    err = rel_norm(host(lam), lam_ref)
    say(f"[mixed] its {info['iters']} reported {info['rel_res']:.2e} oracle residual {true_res:.2e} err vs FP64 {err:.2e}")
    assert info["status"] == 0 and true_res <= 1e-8
    # the FP32 preconditioner is applied inside FP64 FGMRES: the error is set by the tolerance
    assert err <= 1e-5


@pytest.mark.gpu
def test_edge_cases():
    prob, orc, s = setup("box16")
    import torch

    n = orc.mesh.ntrace
    b = torch.zeros(n, dtype=torch.float64, device="cuda")
    lam = torch.ones(n, dtype=torch.float64, device="cuda")
    info = s.solve(b, lam, rtol=1e-8)
    assert info["status"] == 0 and info["iters"] == 0 and float(lam.abs().max()) == 0.0
    rng = np.random.default_rng(9)
    b = dev(rng.standard_normal(n))
    lam = torch.zeros(n, dtype=torch.float64, device="cuda")
    info = s.solve(b, lam, rtol=1e-12, maxit=1)
    assert info["status"] == 1 and info["iters"] == 1
    # restarting from the returned iterate continues to converge
    info2 = s.solve(b, lam, rtol=1e-8, maxit=200)
    assert info2["status"] == 0
    # restart length 1 still converges (slowly), the status is reported
    from gpu_common import params_for

    s.set_params(params_for(prob, restart=5))
    lam.zero_()
    info3 = s.solve(b, lam, rtol=1e-8, maxit=400)
    assert info3["status"] == 0 and info3["restarts"] >= 1
    # cycles longer than 31 steps use three-pass Gram-Schmidt (and a conditional second pass from
    # step 32 on) instead of the delayed reorthogonalisation: run 36 steps without a tolerance
    s.set_params(params_for(prob, restart=40))
    lam.zero_()
    info4 = s.solve(b, lam, rtol=0.0, maxit=36)
    y = torch.empty_like(b)
    s.trace_apply(lam, y)
    res4 = float(torch.linalg.norm(b - y) / torch.linalg.norm(b))
    say(f"[restart 40] 36 steps: true residual {res4:.1e}")
    assert info4["iters"] == 36 and res4 <= 1e-11
    s.set_params(params_for(prob))
    # a tolerance below the rounding floor of the residual: the solve stops once two restart cycles
    # in a row leave the true residual where it was, and says so
    from paper_2210_11797_amd import HYB_STAGNATED

    lam.zero_()
    info5 = s.solve(b, lam, rtol=1e-20, maxit=2000)
    say(f"[stagnation] rtol 1e-20: status {info5['status']} after {info5['iters']} iterations, "
        f"residual {info5['rel_res']:.1e}")
    assert info5["status"] == HYB_STAGNATED and info5["iters"] < 2000 and info5["rel_res"] <= 1e-14
    # bad arguments are rejected, not crashed on
    with pytest.raises(RuntimeError):
        s.trace_apply(b, b)


WIDE = {
    # 32768 columns on the fine level: its sweeps run one lane per column (residual and column solve
    # fused); the coarse level of 8192 columns takes the cyclic-reduction sweeps
    "wide256": dict(nx=256, ny=128, nlev=4, dx=5e3, dz=250.0, mg_levels=2, perturb=0.05),
    # a coarsest level of 32768 columns: its Chebyshev steps run one lane per column as well
    "wide_coarsest": dict(nx=256, ny=256, nlev=2, dx=5e3, dz=250.0, mg_levels=2, perturb=0.05),
}


@pytest.mark.gpu
def test_zero_gamma_switch_leaves_the_smoother_sweeps():
    """Failure injection from the host: with Gamma taken as zero the coarse correction adds nothing,
    so the two-level cycle is bit for bit its LineSmooth sweeps (the smoother-only configuration
    with the same sweeps), and FGMRES still converges, with more iterations."""
    import torch

    from paper_2210_11797_amd import HYB_DEBUG_ZERO_GAMMA

    prob = make_box(**CASES["ragged"])
    s = make_solver(prob)
    r = dev(np.random.default_rng(8).standard_normal(s.ntrace))
    z = {}
    for name, kw in (("zero_gamma", dict(debug=HYB_DEBUG_ZERO_GAMMA)), ("smoother_only", dict(coarse_mode=1)),
                     ("two_level", {})):
        p = s.params
        p.debug, p.coarse_mode = kw.get("debug", 0), kw.get("coarse_mode", 0)
        s.set_params(p)
        z[name] = torch.empty_like(r)
        s.precondition(r, z[name])
    assert torch.equal(z["zero_gamma"], z["smoother_only"])
    assert not torch.equal(z["zero_gamma"], z["two_level"])
    its = {}
    for flag in (0, HYB_DEBUG_ZERO_GAMMA):
        p = s.params
        p.debug, p.coarse_mode = flag, 0
        s.set_params(p)
        its[flag] = s.solve(r, torch.zeros_like(r), rtol=1e-8, maxit=3000)["iters"]
    say(f"[zero gamma] FGMRES iterations: two-level {its[0]}, Gamma = 0 {its[HYB_DEBUG_ZERO_GAMMA]}")
    assert its[HYB_DEBUG_ZERO_GAMMA] > its[0]
    s.close()



@pytest.mark.gpu
@pytest.mark.parametrize("mesh", ["box_tiles", "sphere_c8x6"])
@pytest.mark.parametrize("precision", [0, 1])
def test_paired_restriction_matches_the_children_map(mesh, precision):
    """Where the children of every coarse column are two pairs of adjacent columns (the box and the
    cubed sphere number them so) the multigrid restriction loads each pair as one vector; with
    HYB_DEBUG_UNPAIRED_RESTRICT it reads every child through the children map.  Same arithmetic in
    the same order: the preconditioner and whole solves agree bit for bit, in both precisions."""
    import torch

    from paper_2210_11797_amd import HYB_DEBUG_UNPAIRED_RESTRICT
    from synth import make_sphere

    if mesh == "box_tiles":
        prob = make_box(nx=24, ny=20, nlev=6, dx=5e3, dz=500.0, mg_levels=3, perturb=0.02)
    else:
        prob = make_sphere(8, 6, mg_levels=3, perturb=0.05)
    s = make_solver(prob, precision=precision)
    r = dev(np.random.default_rng(11).standard_normal(s.ntrace))
    z, lam, its = {}, {}, {}
    for flag in (0, HYB_DEBUG_UNPAIRED_RESTRICT):
        p = s.params
        p.debug = flag
        s.set_params(p)
        z[flag] = torch.empty_like(r)
        s.precondition(r, z[flag])
        lam[flag] = torch.zeros_like(r)
        its[flag] = s.solve(r, lam[flag], rtol=1e-10, maxit=400)["iters"]
    say(f"[paired restriction] {mesh} precision {precision}: {its[0]} iterations both ways")
    assert torch.equal(z[0], z[HYB_DEBUG_UNPAIRED_RESTRICT])
    assert its[0] == its[HYB_DEBUG_UNPAIRED_RESTRICT] and torch.equal(lam[0], lam[HYB_DEBUG_UNPAIRED_RESTRICT])
    s.close()

PATCH = {
    "ragged": dict(nx=12, ny=10, nlev=5, dx=7e3, dy=5e3, dz=400.0, mg_levels=2, perturb=0.1),
    "tiles_stretched": dict(nx=24, ny=20, nlev=12, dx=5e3, ztop=6e3, stretch="quadratic", mg_levels=3,
                            perturb=0.2, theta_col_perturb=0.05),
}


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(PATCH))
@pytest.mark.parametrize("precision", [0, 1])
def test_precondition_patch_cached_smoother(name, precision):
    """LineSmooth with the tridiagonal column matrices cached per 2x2 patch (the mean of the
    patch's S^zz, future work of Sec. 4.2) against the oracle's variant: the preconditioner at
    100 eps cond(H) (FP64), and the solve (to 1e-14, or its rounding floor below 1e-13) against the
    direct solution to 1e-10 in both precisions."""
    import torch

    prob = make_box(**PATCH[name])
    say(f"[setup] patch-cached smoother {name} precision {precision}")
    orc = OracleProblem(prob, with_mixed=False, smoother_patch=True)
    s = make_solver(prob, smoother_patch=1, precision=precision)
    rng = np.random.default_rng(6)
    r = rng.standard_normal(orc.mesh.ntrace)
    ref = orc.pc(r)
    cond_h = np.linalg.cond(orc.H.toarray())
    tol = max(1e-12, 100 * np.finfo(float).eps * cond_h)
    moved = rel_max(OracleProblem(prob, with_mixed=False).pc(r), ref)
    if precision == 0:
        z = torch.empty(orc.mesh.ntrace, dtype=torch.float64, device="cuda")
        s.precondition(dev(r), z)
        err = rel_max(host(z), ref)
        say(f"[precondition, patch] {name}: rel err {err:.2e} (tol {tol:.1e}; the variant moves z by {moved:.1e})")
        assert err <= tol and moved > 10 * tol
    r_ub, r_pi = make_rhs(prob, 3)
    ruc, rpc = cells_from_soa(r_ub, r_pi)
    b = torch.empty(orc.mesh.ntrace, dtype=torch.float64, device="cuda")
    s.condense(dev(r_ub), dev(r_pi), b)
    lam_ref = orc.hyb.solve_direct(ruc, rpc)[0]
    lam = torch.zeros_like(b)
    info = s.solve(b, lam, rtol=1e-14, maxit=400)
    err = rel_norm(host(lam), lam_ref)
    say(f"[solve, patch] {name} precision {precision}: {info['iters']} iterations, residual {info['rel_res']:.1e}, "
        f"lambda err {err:.1e}")
    assert info["rel_res"] <= 1e-13 and err <= 1e-10
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(WIDE))
def test_precondition_large_levels(name):
    """hyb_precondition on meshes whose multigrid levels have more than 16384 columns, against the
    oracle, to 100 eps cond(H) (cond by the 1-norm estimate of H and H^-1)."""
    import scipy.sparse.linalg as spla
    import torch

    say(f"[setup] case {name}: {WIDE[name]}")
    prob = make_box(**WIDE[name])
    orc = OracleProblem(prob)
    s = make_solver(prob)
    r = np.random.default_rng(3).standard_normal(orc.mesh.ntrace)
    z = torch.empty(orc.mesh.ntrace, dtype=torch.float64, device="cuda")
    s.precondition(dev(r), z)
    ref = orc.pc(r)
    err = rel_max(host(z), ref)
    H = orc.H.tocsc()
    lu = spla.splu(H)
    hinv = spla.LinearOperator(H.shape, matvec=lu.solve, rmatvec=lambda v: lu.solve(v, trans="T"))
    cond_h = spla.onenormest(H) * spla.onenormest(hinv)
    tol = 100 * np.finfo(float).eps * cond_h
    say(f"[precondition] {name}: rel err {err:.2e} (cond(H) ~ {cond_h:.1e}, tol {tol:.1e})")
    assert err <= tol
    s.close()


@pytest.mark.gpu
def test_precondition_chunked_restriction():
    """hyb_precondition where the finest restriction gives each thread a chunk of levels (1M cells:
    4096 coarse columns x 67 levels, chunks of 2 with a ragged last one), against the oracle.  The
    tolerance is 100 eps cond(H) with cond(H) taken on a 16x16 box of the same spacings and levels:
    on a periodic box H splits into horizontal Fourier modes, the 16x16 box holds the modes of the
    extreme eigenvalues (zero and Nyquist wavenumbers) of the 128x128 one, and a factor 2 covers the
    5 % perturbation of the mesh."""
    import scipy.sparse.linalg as spla
    import torch

    spec = dict(nx=128, ny=128, nlev=67, dx=5e3, dz=250.0, mg_levels=2, perturb=0.05)
    say(f"[setup] chunked restriction: {spec}")
    proxy = OracleProblem(make_box(**dict(spec, nx=16, ny=16)))
    H = proxy.H.tocsc()
    lu = spla.splu(H)
    hinv = spla.LinearOperator(H.shape, matvec=lu.solve, rmatvec=lambda v: lu.solve(v, trans="T"))
    cond_h = spla.onenormest(H) * spla.onenormest(hinv)
    prob = make_box(**spec)
    orc = OracleProblem(prob)
    s = make_solver(prob)
    r = np.random.default_rng(5).standard_normal(orc.mesh.ntrace)
    z = torch.empty(orc.mesh.ntrace, dtype=torch.float64, device="cuda")
    s.precondition(dev(r), z)
    err = rel_max(host(z), orc.pc(r))
    tol = 2 * 100 * np.finfo(float).eps * cond_h
    say(f"[precondition] chunked restriction: rel err {err:.2e} (cond(H) ~ {cond_h:.1e}, tol {tol:.1e})")
    assert err <= tol
    s.close()
