"""Benchmark: time-to-1e-8 of one hybridised trace solve on one MI355X.

One step = condense the right-hand side (B_lambda = C^T A^-1 R_X), FGMRES with the two-level
preconditioner from lambda = 0 to ||B - S lambda|| / ||B|| <= 1e-8, and recover (u_b, Pi), on the
periodic 256 x 256 x 64 box (dx = 5 km, dz = 250 m, dt = 600 s; 4.19M cells, 12.6M trace
unknowns).  Inputs are synthetic (seeded N(0,1) right-hand sides) and resident in HBM before the
timed region; operator setup (assembly, condensation, multigrid setup) is done once, outside.

Prints one JSON line (rank 0) with the time per solve (a timed region without events), the
algorithmic HBM bandwidth of the solve, the roofline of the dominant kernel (its launches timed with
HIP events on the solver's stream over a second run of the same solves) and the CPU oracle.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
FAMILIES = ("smooth_rows", "smooth_rows0", "thomas", "trace_apply", "mg_smooth", "restrict", "prolong", "krylov",
            "cell_solve", "nn")
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
# algorithmic flops of the order-1 condensation per cell: elimination of the 44 x 44 block without
# pivoting (2/3 n^3) and of its 24 right-hand sides (forward and back substitution, 2 n^2 each)
P1_CONDENSE_FLOPS = 2.0 / 3.0 * 44**3 + 2 * 44**2 * 24
# algorithmic HBM bytes of the FP64 condensation by the block structure per cell: the 748 entries
# of A_K it uses (twelve 3x3 velocity blocks, G, D, P), C_F and K_F (24 + 24), S_K written (576)
# and the 748 cell factors written
P1_STRUCT_BYTES = 8 * (748 + 48 + 576 + 748)


def coarsest_desc(args):
    kind = "block-Jacobi sweeps" if args.coarse_jacobi else "Chebyshev steps over block Jacobi on [0.02, 2]"
    return f"{args.coarse_sweeps} {kind}"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def setup_solver(prob, precision, **kw):
    import numpy as np
    import torch

    from paper_2210_11797_amd import HybSolver, Params, levels_of

    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    params = Params(dt=prob.dt, tau_u=prob.tau_u, tau_rho=prob.tau_rho, tau_theta=prob.tau_theta, cp=prob.cp,
                    rd=prob.rd, precision=precision, **kw)
    s = HybSolver(prob.nlev, levels_of(prob), prob.dx, prob.dy, prob.dz, params)
    s.assemble_local(d(prob.theta_w), d(prob.exner_hat_w), d(prob.exner_c), d(prob.rho_c))
    s.condense()
    torch.cuda.synchronize()
    return s


def run_steps(s, rhs, steps, warmup, rtol, profile=False):
    """Times `steps` solves after `warmup`.  profile: False (no events), True (events around
    every kernel family) or a family name (events around that family's launches only)."""
    import torch

    b = torch.empty(s.ntrace, dtype=torch.float64, device="cuda")
    lam = torch.empty_like(b)
    ub = torch.empty(6 * s.ncell, dtype=torch.float64, device="cuda")
    pi = torch.empty(s.ncell, dtype=torch.float64, device="cuda")
    infos = []

    def step(i):
        r_ub, r_pi = rhs[i % len(rhs)]
        s.condense(r_ub, r_pi, b)
        lam.zero_()
        info = s.solve(b, lam, rtol=rtol, maxit=500)
        s.recover(r_ub, r_pi, lam, ub, pi)
        return info

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    if isinstance(profile, str):
        s.profile_family(profile)
    elif profile:
        s.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        infos.append(step(i))
        log(f"step {i}: iters {infos[-1]['iters']} rel_res {infos[-1]['rel_res']:.2e}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fams = {}
    if profile:
        for f in ([profile] if isinstance(profile, str) else FAMILIES):
            fams[f] = s.profile_read(f)
        s.profile(False)
    return (t1 - t0) / steps, infos, fams


def measured_traffic(nx, nlev):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter summary,
    or None when that summary was taken on another workload or the kernel source has changed."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"k_smooth_rows_box{nx}x{nx}x{nlev}.md")
    src = os.path.join(ROOT, "paper_2210_11797_amd", "csrc", "solve.hip")
    if not os.path.exists(path):
        return None
    fields = dict(ln.split(": ", 1) for ln in open(path).read().splitlines()
                  if ln.startswith(("traffic_bytes_per_launch:", "source_sha256:")))
    if fields.get("source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return float(fields["traffic_bytes_per_launch"])


def algorithmic_bytes(ntr, ncell, ncol, nlev, its, fams, steps):
    """Bytes the method must move per solve (FP64): every launch counted by what its definition
    reads and writes once (operator entries, vectors), reuse through caches not counted."""
    nz = (nlev + 1) * ncol
    per = {
        "smooth_rows": 14 * 8 * ntr,                 # S row (11), B, lambda_in, R or lambda_out
        "smooth_rows0": 3 * 8 * (ntr - nz),          # B, diag(S^hh), lambda_out on vertical facets
        "thomas": (40 + 2 * 48) / 3 * nz,            # R or B, 3 factors, lambda_in (not on zero sweep), out
        "trace_apply": 13.5 * 8 * ntr,               # S row, x, (b), y
        "prolong": 16 * ntr + 8 * ncell,             # lambda read/write, dPi
    }
    # V-cycle per launch family: mg_smooth launches split across levels; count per cycle
    total = 0.0
    for f, b in per.items():
        total += fams[f][0] / steps * b
    lev_cells = [ncell / 4**l for l in range(4)]
    cycles = fams["smooth_rows0"][0] / steps
    vcycle = sum(c * 8 * ((5 + 10 + 10) if i < 3 else (5 + 10 + 10)) for i, c in enumerate(lev_cells))
    vcycle += sum(c * 8 * 9.25 for c in lev_cells[:3])  # residual + restriction to the coarse level
    vcycle += ncell * 8 * 8                               # trace residual restriction with Gamma
    total += cycles * vcycle
    for it_count in its:
        for j in range(it_count):
            # Gram-Schmidt with delayed reorthogonalisation: the reduction pass reads V_0..V_{j+1},
            # the update pass reads them and writes V_j and V_{j+1}
            total += 8 * ntr * ((j + 2) + (j + 4)) / len(its)
        total += 8 * ntr * (it_count + 2) / len(its)                # solution update
        total += 8 * ntr * 5 / len(its)                             # ||b||, ||lambda_0||, r_0 = b, ||r_0||
    total += ncell * 8 * (49 + 7 + 6) + 8 * 9 * ntr / 3            # condense RHS + facet gather
    total += ncell * 8 * (49 + 7 + 6 + 6 + 7)                      # recover
    return total


def cpu_baseline(prob, coarse_sweeps, coarse_jacobi, seeds=(0, 1, 2, 3, 4), threads=1):
    """The oracle's hybridised FGMRES solve (condense RHS + FGMRES to 1e-8 with the two-level
    preconditioner + recover) on ``prob``, ``threads`` BLAS threads (SciPy's sparse kernels are single
    threaded): the median over the seeds of the seconds per solve, setup excluded."""
    from threadpoolctl import threadpool_limits

    from oracle.problem import OracleProblem, cells_from_soa
    from synth import make_rhs

    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        orc = OracleProblem(prob, mg_coarse_sweeps=coarse_sweeps,
                            mg_coarse_cheb=None if coarse_jacobi else (0.02, 2.0), log=log)
        t_setup = time.perf_counter() - t0
        times, its = [], []
        for sd in seeds:
            ruc, rpc = cells_from_soa(*make_rhs(prob, sd))
            t0 = time.perf_counter()
            B = orc.hyb.rhs(ruc, rpc)
            x, hist, it, conv = orc.solve_fgmres(B, rtol=1e-8)
            orc.hyb.recover(x, ruc, rpc)
            times.append(time.perf_counter() - t0)
            its.append(it)
            log(f"cpu baseline: {prob.nx}x{prob.ny}x{prob.nlev} seed {sd}: {times[-1]:.2f} s, {it} iterations")
    return dict(median_s=float(sorted(times)[len(times) // 2]), times=times, setup_s=t_setup, iters=its,
                ncell=prob.ncell)


def splu_scaling(nxs, dx, dz, dt, nlev_of, cap_s):
    """(A) the sparse direct solve of the unhybridised 2x2 system (SuperLU, one core) on growing boxes
    of the workload's physics, each in a subprocess limited to cap_s seconds; stops at the first box
    that does not finish (time or memory)."""
    import subprocess

    out = []
    for nx in nxs:
        nlev = nlev_of(nx)
        code = (
            "import sys, time, resource; sys.path.insert(0, %r)\n"
            "from oracle.local import local_matrices\nfrom oracle.mesh import BoxMesh\n"
            "from oracle.mixed import MixedSystem\nfrom oracle.problem import cells_from_soa\n"
            "from synth import make_box, make_rhs\nimport scipy.sparse.linalg as spla\n"
            "p = make_box(nx=%d, ny=%d, nlev=%d, dx=%r, dz=%r, dt=%r, mg_levels=1)\n"
            "m = BoxMesh(p.nx, p.ny, p.nlev, p.dx, p.dy, p.z)\nmx = MixedSystem(m, local_matrices(m, p), p)\n"
            "rhs = mx.rhs(*cells_from_soa(*make_rhs(p, 0)))\nt = time.perf_counter()\n"
            "lu = spla.splu(mx.matrix)\nt1 = time.perf_counter()\nx = lu.solve(rhs)\nt2 = time.perf_counter()\n"
            "print(p.ncell, mx.matrix.shape[0], t1 - t, t2 - t1, resource.getrusage(resource.RUSAGE_SELF).ru_maxrss)\n"
        ) % (ROOT, nx, nx, nlev, dx, dz, dt)
        try:
            res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=cap_s)
        except subprocess.TimeoutExpired:
            out.append(dict(box=f"{nx}x{nx}x{nlev}", status=f"did not finish in {cap_s} s"))
            log(f"splu: {nx}x{nx}x{nlev} did not finish in {cap_s} s")
            break
        if res.returncode != 0:
            out.append(dict(box=f"{nx}x{nx}x{nlev}", status=f"failed ({res.stderr.strip()[-200:]})"))
            break
        ncell, n, tf, ts, rss = res.stdout.split()
        out.append(dict(box=f"{nx}x{nx}x{nlev}", ncell=int(ncell), unknowns=int(n), factor_s=float(tf),
                        solve_s=float(ts), max_rss_gb=int(rss) / 1e6))
        log(f"splu: {out[-1]}")
    return out


def learned_leg(args, prob, s, rhs, sec_plain, dx, dz, dt):
    """Train the learned stage on a smaller box of the same physics (the network is local and
    translation-equivariant, so its weights carry over), outside the timed region; then time the
    solves with the stage on the benchmark box."""
    import numpy as np
    import torch

    from paper_2210_11797_amd import learned
    from synth import make_box, make_rhs

    nt = args.train_nx
    tprob = make_box(nx=nt, ny=nt, nlev=args.nlev, dx=dx, dz=dz, dt=dt, mg_levels=4)
    ts = setup_solver(tprob, 0, mg_coarse_sweeps=args.coarse_sweeps, mg_coarse_cheb=0 if args.coarse_jacobi else 1)
    ts.nn_set_weights(learned.init_params(16, seed=0))
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    t0 = time.perf_counter()
    bl = []
    for sd in range(32):
        r_ub, r_pi = make_rhs(tprob, 20000 + sd)
        b = torch.empty(ts.ntrace, dtype=torch.float64, device="cuda")
        ts.condense(d(r_ub), d(r_pi), b)
        bl.append(b)
    X, R = learned.generate_pairs(ts, bl, steps=8)
    npairs = int(X.shape[0])
    hist = learned.train(ts, X, R, steps=args.train_steps, batch=8, lr=2e-3, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    w = ts.nn_get_weights()
    ts.close()
    del X, R, bl
    s.nn_set_weights(w)
    p = s.params
    p.learned = 1
    s.set_params(p)
    lsec, linfos, lfams = run_steps(s, rhs, args.steps, args.warmup, args.rtol, profile="nn")
    p.learned = 0
    s.set_params(p)
    nn_launches, nn_ms = lfams["nn"]
    return dict(sec_per_solve=lsec, iters=[i["iters"] for i in linfos],
                corrections_kept=[i["iters"] - i["fallbacks"] for i in linfos],
                rel_res=max(i["rel_res"] for i in linfos), speedup_vs_fp64=sec_plain / lsec,
                stage_ms_per_call=nn_ms / max(nn_launches, 1),
                training=dict(box=f"{nt}x{nt}x{args.nlev}", pairs=npairs, steps=args.train_steps,
                              batch=8, final_energy_loss=float(np.mean(hist[-50:])), seconds=train_s))


def configs_leg(args, prob, rhs):
    """The paper's solver configurations on the benchmark box, by time-to-1e-8 and iterations: the
    hybridised single-level method (Configuration 2: FGMRES preconditioned by 1, 2 or 3 LineSmooth
    sweeps), FGMRES on the unhybridised system with the approximate-Schur preconditioner
    (Configuration 1, the paper's baseline) and the two-level cycle with its coarse pressure system solved by BiCGStab + V-cycle to
    1e-14 or 1e-2 (Configurations 3a, 3b) against the two-level cycle with one V-cycle
    (Configuration 3c, the headline form), and the relaxation factor omega of the two-level cycle
    from 0.3 to 0.9 (the paper's parameter study)."""
    import torch

    from paper_2210_11797_amd import PREC_FP64, PREC_MIXED

    out = {"single_level": {}, "omega_two_level": {}}

    def one(s, maxit):
        b = torch.empty(s.ntrace, dtype=torch.float64, device="cuda")
        lam = torch.zeros_like(b)
        s.condense(rhs[0][0], rhs[0][1], b)
        s.solve(b, lam, rtol=args.rtol, maxit=maxit)  # warm-up
        lam.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = s.solve(b, lam, rtol=args.rtol, maxit=maxit)
        torch.cuda.synchronize()
        return dict(sec_per_solve=time.perf_counter() - t0, iters=info["iters"], rel_res=info["rel_res"],
                    status=info["status"])

    for n in (1, 2, 3):
        s = setup_solver(prob, 0, coarse_mode=1, n_pre=n, n_post=0, mg_coarse_sweeps=args.coarse_sweeps)
        out["single_level"][f"{n}_sweeps"] = r = one(s, 6000)
        log(f"configuration 2 ({n} sweeps): {r['sec_per_solve'] * 1e3:.0f} ms, {r['iters']} iterations")
        s.close()
    # Configuration 1: FGMRES on the unhybridised system with the approximate-Schur preconditioner,
    # from the same broken right-hand side (the mixed right-hand side assembled inside the timing)
    s = setup_solver(prob, 0, mg_coarse_sweeps=args.coarse_sweeps)
    bm = torch.empty(s.nmixed, dtype=torch.float64, device="cuda")
    xm = torch.zeros_like(bm)
    s.mixed_rhs(rhs[0][0], rhs[0][1], bm)
    s.mixed_solve(bm, xm, rtol=args.rtol, maxit=1000)  # warm-up (allocates the mixed Krylov basis)
    xm.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.mixed_rhs(rhs[0][0], rhs[0][1], bm)
    info = s.mixed_solve(bm, xm, rtol=args.rtol, maxit=1000)
    torch.cuda.synchronize()
    out["configuration_1"] = r = dict(sec_per_solve=time.perf_counter() - t0, iters=info["iters"],
                                      rel_res=info["rel_res"], status=info["status"])
    log(f"configuration 1 (approximate Schur, unhybridised): {r['sec_per_solve'] * 1e3:.1f} ms, {r['iters']} iterations, "
        f"status {r['status']}")
    del bm, xm
    s.close()
    for name, crt in (("3a", 1e-14), ("3b", 1e-2)):
        s = setup_solver(prob, 0, coarse_mode=2, coarse_rtol=crt, mg_coarse_sweeps=args.coarse_sweeps)
        out[f"configuration_{name}"] = r = one(s, 1000)
        log(f"configuration {name} (BiCGStab + V-cycle coarse solve to {crt:.0e}): {r['sec_per_solve'] * 1e3:.1f} ms, "
            f"{r['iters']} iterations")
        s.close()
    # LineSmooth with the column matrices cached per 2x2 patch of columns (future work of Sec. 4.2):
    # a quarter of the factor reads of the column solve, against what it costs in iterations
    out["smoother_patch"] = {}
    for name, prec in (("fp64", PREC_FP64), ("mixed", PREC_MIXED)):
        for patch in (0, 1):
            s = setup_solver(prob, prec, smoother_patch=patch, mg_coarse_sweeps=args.coarse_sweeps)
            out["smoother_patch"][f"{name}_{'patch' if patch else 'per_column'}"] = r = one(s, 1000)
            log(f"configuration 3c {name}, column matrices {'per 2x2 patch' if patch else 'per column'}: "
                f"{r['sec_per_solve'] * 1e3:.1f} ms, {r['iters']} iterations")
            s.close()
    for om in (0.3, 0.5, 0.6, 0.7, 0.8, 0.9):
        s = setup_solver(prob, 0, omega=om, mg_coarse_sweeps=args.coarse_sweeps)
        out["omega_two_level"][f"{om:.1f}"] = r = one(s, 1000)
        log(f"configuration 3c, omega {om:.1f}: {r['sec_per_solve'] * 1e3:.1f} ms, {r['iters']} iterations, "
            f"status {r['status']}")
        s.close()
    torch.cuda.empty_cache()
    return out


def appendix_b_leg(args, prob, rhs):
    """The paper's solver-parameter study (its appendix on solver parameters) on the benchmark box:
    time-to-1e-8 and iterations of FGMRES on the unhybridised system (Configuration 1) over the
    pressure multigrid's relaxation factor omega_p = 0.3 ... 1.0 and 1-2 pre- / post-smoothing
    steps, of the hybridised single-level method (Configuration 2) over the
    smoother's relaxation factor omega = 0.3 ... 1.0 and 1, 2, 3 sweeps, and of the two-level cycle
    (Configuration 3c; pressure V-cycle fixed) over omega and 1-3 pre- / 1-2 post-smoothing steps.
    A run that has not reached the tolerance within its iteration cap (300 for Configuration 1, 3000 for Configuration 2,
    300 for 3c) counts as not converged (status 1)."""
    import torch

    omegas = (0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0)
    out = {"configuration_1": {}, "configuration_2": {}, "configuration_3c": {}}

    def one(s, maxit):
        b = torch.empty(s.ntrace, dtype=torch.float64, device="cuda")
        lam = torch.zeros_like(b)
        s.condense(rhs[0][0], rhs[0][1], b)
        s.solve(b, lam, rtol=args.rtol, maxit=2)  # allocates the Krylov basis outside the timing
        lam.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = s.solve(b, lam, rtol=args.rtol, maxit=maxit)
        torch.cuda.synchronize()
        return dict(sec_per_solve=time.perf_counter() - t0, iters=info["iters"], rel_res=info["rel_res"],
                    status=info["status"])

    bm = None
    for mg_pre in (1, 2):
        for mg_post in (1, 2):
            row = out["configuration_1"][f"{mg_pre}_pre_{mg_post}_post"] = {}
            for om in omegas:
                s = setup_solver(prob, 0, omega_p=om, mg_pre=mg_pre, mg_post=mg_post,
                                 mg_coarse_sweeps=args.coarse_sweeps)
                if bm is None:
                    bm = torch.empty(s.nmixed, dtype=torch.float64, device="cuda")
                xm = torch.zeros_like(bm)
                s.mixed_rhs(rhs[0][0], rhs[0][1], bm)
                s.mixed_solve(bm, xm, rtol=args.rtol, maxit=2)  # allocates the Krylov bases
                xm.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = s.mixed_solve(bm, xm, rtol=args.rtol, maxit=300)
                torch.cuda.synchronize()
                row[f"{om:.1f}"] = r = dict(sec_per_solve=time.perf_counter() - t0, iters=info["iters"],
                                            rel_res=info["rel_res"], status=info["status"])
                s.close()
                del xm
                log(f"appendix B, configuration 1, pressure MG {mg_pre} pre {mg_post} post, omega_p {om:.1f}: "
                    f"{r['sec_per_solve'] * 1e3:.1f} ms, {r['iters']} iterations, status {r['status']}")
    del bm
    for n in (1, 2, 3):
        row = out["configuration_2"][f"{n}_sweeps"] = {}
        for om in omegas:
            s = setup_solver(prob, 0, coarse_mode=1, n_pre=n, n_post=0, omega=om,
                             mg_coarse_sweeps=args.coarse_sweeps)
            row[f"{om:.1f}"] = r = one(s, 3000)
            s.close()
            log(f"appendix B, configuration 2, {n} sweep(s), omega {om:.1f}: {r['sec_per_solve'] * 1e3:.0f} ms, "
                f"{r['iters']} iterations, status {r['status']}")
    for n_pre in (1, 2, 3):
        for n_post in (1, 2):
            row = out["configuration_3c"][f"{n_pre}_pre_{n_post}_post"] = {}
            for om in omegas:
                s = setup_solver(prob, 0, n_pre=n_pre, n_post=n_post, omega=om,
                                 mg_coarse_sweeps=args.coarse_sweeps)
                row[f"{om:.1f}"] = r = one(s, 300)
                s.close()
                log(f"appendix B, configuration 3c, {n_pre} pre {n_post} post, omega {om:.1f}: "
                    f"{r['sec_per_solve'] * 1e3:.1f} ms, {r['iters']} iterations, status {r['status']}")
    torch.cuda.empty_cache()
    return out


def sphere_leg(args):
    """The extruded cubed sphere (C192 x 30 quadratic layers to 30 km, dt = 1800 s, rotating, the
    Gaussian pressure bump): time-to-1e-8 of the plain FP64 solve and of the mixed form, their
    iterations, and the error of the mixed solution against the FP64 one; the same with LineSmooth's
    column matrices cached per 2x2 patch (future work of Sec. 4.2), which on this mesh, unlike the
    uniform box, changes the smoother."""
    import numpy as np
    import torch

    from paper_2210_11797_amd import PREC_FP64, PREC_MIXED, Params, solver_for
    from synth import make_rhs_sphere, make_sphere

    prob = make_sphere(args.sphere_n, args.sphere_nlev, dt=args.sphere_dt, mg_levels=4)
    log(f"sphere: C{args.sphere_n} x {args.sphere_nlev}, {prob.ncell} cells, {prob.ntrace} trace unknowns")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    rhs = [tuple(d(a) for a in make_rhs_sphere(prob, sd)) for sd in range(3)]
    out, lam0 = {}, {}
    for name, prec, patch in (("fp64", PREC_FP64, 0), ("mixed", PREC_MIXED, 0), ("fp64_patch", PREC_FP64, 1),
                              ("mixed_patch", PREC_MIXED, 1)):
        params = Params(dt=prob.dt, tau_u=prob.tau_u, tau_rho=prob.tau_rho, tau_theta=prob.tau_theta, cp=prob.cp,
                        rd=prob.rd, precision=prec, omega_rot=prob.omega_rot, mg_coarse_sweeps=args.coarse_sweeps,
                        mg_coarse_cheb=0 if args.coarse_jacobi else 1, smoother_patch=patch)
        s = solver_for(prob, params)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.assemble_local(d(prob.theta_w), d(prob.exner_hat_w), d(prob.exner_c), d(prob.rho_c))
        s.condense()
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        sec, infos, _ = run_steps(s, rhs, 3, 1, args.rtol, profile=False)
        rec = dict(sec_per_solve=sec, iters=[i["iters"] for i in infos], rel_res=max(i["rel_res"] for i in infos),
                   setup_s=setup)
        if name == "fp64":
            _, _, fams = run_steps(s, rhs, 3, 0, args.rtol, profile=True)
            nbytes = algorithmic_bytes(s.ntrace, s.ncell, s.ncol, prob.nlev, rec["iters"], fams, 3)
            rec["hbm_gbs_algorithmic"] = nbytes / sec / 1e9
            rec["bytes_per_solve"] = nbytes
        b = torch.empty(s.ntrace, dtype=torch.float64, device="cuda")
        lam = torch.zeros_like(b)
        s.condense(rhs[0][0], rhs[0][1], b)
        s.solve(b, lam, rtol=args.rtol, maxit=500)
        lam0[name] = lam
        out[name] = rec
        log(f"sphere {name}: {sec * 1e3:.1f} ms per solve, iters {rec['iters']}, setup {setup * 1e3:.0f} ms")
        s.close()
        del s
        torch.cuda.empty_cache()
    for name in ("mixed", "fp64_patch", "mixed_patch"):
        out[name]["speedup_vs_fp64"] = out["fp64"]["sec_per_solve"] / out[name]["sec_per_solve"]
        out[name]["lambda_error_vs_fp64"] = float(torch.linalg.norm(lam0[name] - lam0["fp64"]) /
                                                  torch.linalg.norm(lam0["fp64"]))
    return dict(workload=f"cubed sphere C{args.sphere_n} x {args.sphere_nlev} quadratic layers to 30 km, radius "
                         f"6371 km, Omega 7.292e-5/s, dt={args.sphere_dt:.0f}s, RT0/Q0/trace, seeded N(0,1) RHS plus "
                         f"the Gaussian pressure bump, FGMRES(30)+two-level, rtol {args.rtol}",
                ncell=prob.ncell, ntrace=prob.ntrace, forms=out)


def c384_leg(args):
    """The learned stage on the extruded cubed spheres: trained on pairs from plain solves on
    C{sphere_n} x {sphere_nlev} (C192 x 30 by default: 4096 pairs made on the fly from 512
    right-hand sides (drawn on the device) x 8 steps of the plain iteration, kept in a pool of 256 and used by 300 Adam
    steps of batch 8 on the energy loss; BF16 matrix-core training passes), outside the timed
    region; then time-to-1e-8 of the plain FP64 solve and of the solve with the stage on that mesh
    (held-out right-hand sides) and on C{c384_n} x {c384_nlev} (quadratic layers to 30 km, dt =
    900 s, rotating; 61.9M cells), where the mixed form is timed too.  The network is local (a
    3 x 3 x 5 neighbourhood of normalised residuals, 7 x 7 x 13 cells through three layers), so its
    weights carry over between the meshes.  One solver is alive at a time (the C384 FP64 one with
    its FGMRES(30) basis takes ~210 GB)."""
    import numpy as np
    import torch

    from paper_2210_11797_amd import PREC_FP64, PREC_MIXED, Params, learned, solver_for
    from synth import make_rhs_sphere, make_sphere

    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731

    def build(prob, prec):
        params = Params(dt=prob.dt, tau_u=prob.tau_u, tau_rho=prob.tau_rho, tau_theta=prob.tau_theta, cp=prob.cp,
                        rd=prob.rd, precision=prec, omega_rot=getattr(prob, "omega_rot", 0.0),
                        mg_coarse_sweeps=args.coarse_sweeps,
                        mg_coarse_cheb=0 if args.coarse_jacobi else 1)
        sv = solver_for(prob, params)
        sv.assemble_local(d(prob.theta_w), d(prob.exner_hat_w), d(prob.exner_c), d(prob.rho_c))
        sv.condense()
        torch.cuda.synchronize()
        return sv

    def plain_and_learned(s, rhs, w, tag):
        sec, infos, _ = run_steps(s, rhs, 2, 1, args.rtol, profile=False)
        res = dict(fp64=dict(sec_per_solve=sec, iters=[i["iters"] for i in infos],
                             rel_res=max(i["rel_res"] for i in infos)))
        log(f"{tag} fp64: {sec * 1e3:.1f} ms per solve, iters {res['fp64']['iters']}")
        s.nn_set_weights(w)
        p = s.params
        p.learned = 1
        s.set_params(p)
        lsec, linfos, lfams = run_steps(s, rhs, 2, 1, args.rtol, profile=False)
        _, _, lfams = run_steps(s, rhs, 1, 0, args.rtol, profile="nn")
        p.learned = 0
        s.set_params(p)
        nn_launches, nn_ms = lfams["nn"]
        res["learned"] = dict(sec_per_solve=lsec, iters=[i["iters"] for i in linfos],
                              corrections_kept=[i["iters"] - i["fallbacks"] for i in linfos],
                              rel_res=max(i["rel_res"] for i in linfos), speedup_vs_fp64=sec / lsec,
                              stage_ms_per_call=nn_ms / max(nn_launches, 1))
        log(f"{tag} learned: {lsec * 1e3:.1f} ms per solve, iters {res['learned']['iters']}, stage "
            f"{res['learned']['stage_ms_per_call']:.2f} ms per call")
        # the strict judge (a correction kept only if it lowers the residual norm)
        p.learned, p.learned_tau = 1, 1.0
        s.set_params(p)
        ssec, sinfos, _ = run_steps(s, rhs, 2, 1, args.rtol, profile=False)
        p.learned, p.learned_tau = 0, 3.0
        s.set_params(p)
        res["learned_tau1"] = dict(sec_per_solve=ssec, iters=[i["iters"] for i in sinfos],
                                   corrections_kept=[i["iters"] - i["fallbacks"] for i in sinfos],
                                   speedup_vs_fp64=sec / ssec)
        log(f"{tag} learned, tau = 1: {ssec * 1e3:.1f} ms per solve, iters {res['learned_tau1']['iters']}, kept "
            f"{res['learned_tau1']['corrections_kept']}")
        return res

    # training on C192 x 30, pairs on the fly
    tprob = make_sphere(args.sphere_n, args.sphere_nlev, dt=args.sphere_dt, mg_levels=4)
    tmesh = f"C{args.sphere_n} x {args.sphere_nlev} sphere (dt {args.sphere_dt:.0f} s)"
    ts = build(tprob, PREC_FP64)
    ts.nn_set_weights(learned.init_params(16, seed=0))
    # training right-hand sides drawn on the device (the host generator takes ~0.5 s per C192 field):
    # N(0,1) broken velocity and pressure residuals plus the workload's fixed pressure bump
    bump = d(make_rhs_sphere(tprob, 0)[1] - make_rhs_sphere(tprob, 0, bump=0.0)[1]).view(-1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(20000)
    nc = tprob.ncell

    def next_rhs():
        r_ub = torch.randn(6 * nc, generator=gen, dtype=torch.float64, device="cuda")
        r_pi = torch.randn(nc, generator=gen, dtype=torch.float64, device="cuda") + bump
        b = torch.empty(ts.ntrace, dtype=torch.float64, device="cuda")
        ts.condense(r_ub, r_pi, b)
        return b

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist, npairs = learned.train_streaming(ts, next_rhs, npairs=args.train_pairs, pool=256, steps_per_rhs=8, batch=8,
                                           lr=2e-3, updates=args.train_updates, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    w = ts.nn_get_weights()
    log(f"c384: trained on {tmesh}, {npairs} pairs, {len(hist)} updates, {train_s:.1f} s")
    training = dict(mesh=tmesh, pairs=npairs, pool=256, updates=len(hist), batch=8, precision="bf16 mfma",
                    final_energy_loss=float(np.mean(hist[-50:])), seconds=train_s)
    trhs = [tuple(d(a) for a in make_rhs_sphere(tprob, 1000 + sd)) for sd in range(2)]
    c192 = plain_and_learned(ts, trhs, w, f"C{args.sphere_n}")
    ts.close()
    del ts, trhs
    torch.cuda.empty_cache()

    n = args.c384_n
    prob = make_sphere(n, args.c384_nlev, dt=args.c384_dt, mg_levels=4)
    log(f"c384: C{n} x {args.c384_nlev}, {prob.ncell} cells, {prob.ntrace} trace unknowns")
    rhs = [tuple(d(a) for a in make_rhs_sphere(prob, 1000 + sd)) for sd in range(2)]
    s = build(prob, PREC_FP64)
    ws = s.workspace_bytes() / 1e9
    out = plain_and_learned(s, rhs, w, f"C{n}")
    out["workspace_gb"] = ws
    _, infos, fams = run_steps(s, rhs, 2, 0, args.rtol, profile=True)
    nbytes = algorithmic_bytes(s.ntrace, s.ncell, s.ncol, prob.nlev, [i["iters"] for i in infos], fams, 2)
    out["fp64"].update(hbm_gbs_algorithmic=nbytes / out["fp64"]["sec_per_solve"] / 1e9, bytes_per_solve=nbytes)
    s.close()
    del s
    torch.cuda.empty_cache()
    s = build(prob, PREC_MIXED)
    msec, minfos, _ = run_steps(s, rhs, 2, 1, args.rtol, profile=False)
    out["mixed"] = dict(sec_per_solve=msec, iters=[i["iters"] for i in minfos],
                        rel_res=max(i["rel_res"] for i in minfos),
                        speedup_vs_fp64=out["fp64"]["sec_per_solve"] / msec)
    log(f"c384 mixed: {msec * 1e3:.1f} ms per solve, iters {out['mixed']['iters']}")
    s.close()
    del s, rhs
    torch.cuda.empty_cache()
    return dict(workload=f"cubed sphere C{n} x {args.c384_nlev} quadratic layers to 30 km, radius 6371 km, "
                         f"Omega 7.292e-5/s, dt={args.c384_dt:.0f}s, RT0/Q0/trace, seeded N(0,1) RHS plus the "
                         f"Gaussian pressure bump (held-out seeds 1000-1001), FGMRES(30)+two-level, rtol {args.rtol}",
                ncell=prob.ncell, ntrace=prob.ntrace, forms=out, training=training,
                learned_on_training_mesh=dict(mesh=f"C{args.sphere_n} x {args.sphere_nlev}", ncell=tprob.ncell, **c192))


def p1_leg(args):
    """Order 1 (RT1 / DG1 / Q1 trace, 44 x 44 cell blocks) on the 128 x 128 x 32 box (dx = 10 km,
    dz = 500 m): the condensation in FP64 and on MFMA (FP32, BF16 split), and time-to-1e-8 of FGMRES
    with the order-1 two-level preconditioner for each condensed operator, and for the mixed form
    (FP64 operator, FP32 copy of S_K in the preconditioner)."""
    import numpy as np
    import torch

    from paper_2210_11797_amd import HybSolver, Params, PREC_FP64, PREC_MFMA_BF16X, PREC_MFMA_FP32, PREC_MIXED, levels_of
    from synth import make_box, make_rhs_p1

    prob = make_box(nx=args.p1_nx, ny=args.p1_nx, nlev=args.p1_nlev, dx=10e3, dz=500.0, dt=600.0, mg_levels=4)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    rhs = [tuple(d(a) for a in make_rhs_p1(prob, sd)) for sd in range(3)]
    x = d(np.random.default_rng(0).standard_normal(4 * (prob.ncol * (prob.nlev + 1) + 2 * prob.ncol * prob.nlev)))
    out, y64 = {}, None
    for name, prec, dtype in (("fp64", PREC_FP64, "fp64"), ("mixed", PREC_MIXED, "fp64"),
                              ("mfma_fp32", PREC_MFMA_FP32, "fp32"), ("mfma_bf16x", PREC_MFMA_BF16X, "bf16")):
        params = Params(dt=prob.dt, tau_u=prob.tau_u, tau_rho=prob.tau_rho, tau_theta=prob.tau_theta, cp=prob.cp,
                        rd=prob.rd, precision=prec, mg_coarse_sweeps=args.coarse_sweeps,
                        mg_coarse_cheb=0 if args.coarse_jacobi else 1)
        s = HybSolver(prob.nlev, levels_of(prob), prob.dx, prob.dy, prob.dz, params, order=1)
        s.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.assemble_local(d(prob.theta_w), d(prob.exner_hat_w), d(prob.exner_c), d(prob.rho_c))
        s.condense()
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        ncond, cond_ms = s.profile_read("p1_condense")
        nfac, fac_ms = s.profile_read("p1_factor")
        s.profile(False)
        y = torch.empty(s.ntrace, dtype=torch.float64, device="cuda")
        s.trace_apply(x, y)
        if y64 is None:
            y64 = y.clone()
        err = float((y - y64).abs().max() / y64.abs().max())
        b = torch.empty_like(y)
        lam = torch.empty_like(y)
        u = torch.empty(36 * s.ncell, dtype=torch.float64, device="cuda")
        pi = torch.empty(8 * s.ncell, dtype=torch.float64, device="cuda")
        its, res = [], []

        def step(i):
            r_u, r_p = rhs[i % len(rhs)]
            s.condense(r_u, r_p, b)
            lam.zero_()
            info = s.solve(b, lam, rtol=args.rtol, maxit=500)
            s.recover(r_u, r_p, lam, u, pi)
            return info

        step(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(3):
            info = step(i)
            its.append(info["iters"])
            res.append(info["rel_res"])
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / 3
        if ncond:  # dense elimination on matrix cores
            kern_ms = cond_ms
            achieved = P1_CONDENSE_FLOPS * s.ncell / (kern_ms * 1e-3) / 1e12
            roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[dtype], "unit": "TFLOP/s",
                    "frac": achieved / PEAK_TFLOPS[dtype], "kernel": "k_p1_condense_mfma"}
        else:  # FP64 by the block structure, bound by HBM
            kern_ms = fac_ms
            achieved = P1_STRUCT_BYTES * s.ncell / (kern_ms * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": achieved / PEAK_HBM_GBS, "kernel": "k_p1_condense_struct"}
        out[name] = dict(sec_per_solve=sec, iters=its, rel_res=max(res), setup_s=setup, condense_kernel_ms=kern_ms,
                         fp64_factor_ms=fac_ms, s_x_error_vs_fp64=err, roofline=roof)
        unit = roof["unit"]
        log(f"p1 {name}: condense kernel {kern_ms:.2f} ms ({achieved:.2f} {unit}), fp64 factors {fac_ms:.2f} ms, "
            f"solve {sec * 1e3:.1f} ms, iters {its}, S x error vs fp64 {err:.1e}")
        s.close()
        del s
        torch.cuda.empty_cache()
    return dict(workload=f"periodic box {args.p1_nx}x{args.p1_nx}x{args.p1_nlev}, dx=10km, dz=500m, RT1/DG1/Q1 "
                         f"trace (44x44 cell blocks), FGMRES(30)+two-level (DG0 coarse space), rtol {args.rtol}",
                ncell=prob.ncell, ntrace=4 * (prob.ncol * (prob.nlev + 1) + 2 * prob.ncol * prob.nlev),
                condense_flops_per_cell=P1_CONDENSE_FLOPS, struct_bytes_per_cell=P1_STRUCT_BYTES, modes=out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--nlev", type=int, default=64)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-p1", action="store_true")
    ap.add_argument("--no-sphere", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--no-c384", action="store_true")
    ap.add_argument("--appendix-b", action="store_true",
                    help="also run the solver-parameter sweep (Configurations 2 and 3c over omega and smoothing steps)")
    ap.add_argument("--c384-n", type=int, default=384)
    ap.add_argument("--c384-nlev", type=int, default=70)
    ap.add_argument("--c384-dt", type=float, default=900.0)
    ap.add_argument("--train-pairs", type=int, default=4096,
                    help="pairs made on the fly for the learned stage on the spheres")
    ap.add_argument("--train-updates", type=int, default=300, help="Adam steps of that training")
    ap.add_argument("--sphere-n", type=int, default=192)
    ap.add_argument("--sphere-nlev", type=int, default=30)
    ap.add_argument("--sphere-dt", type=float, default=1800.0)
    ap.add_argument("--p1-nx", type=int, default=128)
    ap.add_argument("--p1-nlev", type=int, default=32)
    ap.add_argument("--train-nx", type=int, default=64, help="box on which the learned stage is trained")
    ap.add_argument("--train-steps", type=int, default=300,
                    help="Adam steps of the learned stage (300 generalised better to the 256x256x64 box than 1500)")
    ap.add_argument("--coarse-sweeps", type=int, default=6,
                    help="steps of the coarsest multigrid solve (Chebyshev semi-iteration, or block Jacobi)")
    ap.add_argument("--coarse-jacobi", action="store_true",
                    help="damped block-Jacobi sweeps on the coarsest level instead of the Chebyshev semi-iteration")
    ap.add_argument("--splu-scaling", action="store_true",
                    help="also time SuperLU on the unhybridised system on growing boxes (one core, 170 s cap each)")
    ap.add_argument("--cpu-full-seeds", type=int, default=3, help="seeds of --cpu-baseline-full")
    ap.add_argument("--cpu-baseline-full", action="store_true",
                    help="also time the oracle on the full benchmark workload (--cpu-full-seeds seeds, minutes of "
                         "setup)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB device copy (for scaling HBM counters), outside the timed region")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from synth import make_box, make_rhs

    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", "0")))
    dx, dz, dt = 5e3, 250.0, 600.0
    prob = make_box(nx=args.nx, ny=args.nx, nlev=args.nlev, dx=dx, dz=dz, dt=dt, mg_levels=4)
    log(f"workload: box {args.nx}x{args.nx}x{args.nlev}, {prob.ncell} cells, {prob.ntrace} trace unknowns")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    rhs = []
    for sd in range(5):
        r_ub, r_pi = make_rhs(prob, sd)
        rhs.append((d(r_ub), d(r_pi)))
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1073741824 bytes read, 1073741824 bytes written")
        del src, dst
    t0 = time.perf_counter()
    s = setup_solver(prob, 0, mg_coarse_sweeps=args.coarse_sweeps, mg_coarse_cheb=0 if args.coarse_jacobi else 1)
    setup_s = time.perf_counter() - t0
    log(f"setup (assemble + condense + preconditioner) {setup_s * 1e3:.1f} ms, workspace {s.workspace_bytes() / 1e9:.2f} GB")

    # the headline: timed solves with no events inside; then the same solves again with HIP events
    # (on the solver's stream) around the dominant kernel's launches only, for its average duration,
    # and once more with events around every family for the breakdown and the launch counts
    sec, infos, _ = run_steps(s, rhs, args.steps, args.warmup, args.rtol, profile=False)
    sec_dom, _, dom = run_steps(s, rhs, args.steps, 0, args.rtol, profile="smooth_rows")
    _, _, fams = run_steps(s, rhs, args.steps, 0, args.rtol, profile=True)
    its = [i["iters"] for i in infos]
    ntr, ncell = s.ntrace, s.ncell
    # algorithmic bytes of the dominant kernel: one LineSmooth sweep reads the 11-entry row of S,
    # B and lambda_in and writes lambda_out for every trace row (8 bytes each, FP64)
    # dominant kernel: the LineSmooth residual rows (k_smooth_rows<double,false>), which read the
    # 11-entry row of S, B and lambda_in and write R or lambda_out for every trace row
    ls_launches, ls_ms = dom["smooth_rows"]
    ls_bytes = 14 * 8 * ntr
    ls_avg_ms = ls_ms / max(ls_launches, 1)
    ls_gbs = ls_bytes / (ls_avg_ms * 1e-3) / 1e9
    per_solve_bytes = algorithmic_bytes(ntr, s.ncell, s.ncol, args.nlev, its, fams, args.steps)
    # the implementation-independent count of what the method must move per solve (FP64, per cell:
    # condense RHS and recovery 1.0 KB, per FGMRES iteration Alg. 2 with fused sweeps 1582 B, the
    # matvec 312 B and Gram-Schmidt 48 j + 120 B)
    m_avg = sum(its) / len(its)
    model_bytes = ncell * (1000.0 + 2010.0 * m_avg + 24.0 * m_avg * (m_avg + 1) + 24.0 * (m_avg + 1))
    mixed = None
    if not args.no_mixed:
        sm = setup_solver(prob, 1, mg_coarse_sweeps=args.coarse_sweeps, mg_coarse_cheb=0 if args.coarse_jacobi else 1)
        msec, minfos, _ = run_steps(sm, rhs, args.steps, args.warmup, args.rtol, profile=False)
        mixed = dict(sec_per_solve=msec, iters=[i["iters"] for i in minfos],
                     rel_res=max(i["rel_res"] for i in minfos), speedup_vs_fp64=sec / msec)
        sm.close()

    learned_out = None
    if not args.no_learned:
        learned_out = learned_leg(args, prob, s, rhs, sec, dx, dz, dt)

    configs_out = None
    if not args.no_configs:
        try:
            configs_out = configs_leg(args, prob, rhs)
        except Exception as e:
            log(f"configs leg failed: {e}")
            configs_out = {"error": str(e)}

    appb_out = None
    if args.appendix_b:
        try:
            appb_out = appendix_b_leg(args, prob, rhs)
        except Exception as e:
            log(f"appendix B leg failed: {e}")
            appb_out = {"error": str(e)}

    sphere_out = None
    if not args.no_sphere:
        try:
            sphere_out = sphere_leg(args)
        except Exception as e:  # a failed side leg must not cost the headline line
            log(f"sphere leg failed: {e}")
            sphere_out = {"error": str(e)}

    s.close()
    del s
    torch.cuda.empty_cache()
    c384_out = None
    if not args.no_c384:
        try:
            c384_out = c384_leg(args)
        except Exception as e:
            log(f"c384 leg failed: {e}")
            c384_out = {"error": str(e)}
            torch.cuda.empty_cache()

    p1_out = None
    if not args.no_p1:
        p1_out = p1_leg(args)

    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on the host cores: the paper's parity configuration and a bounded sample of the
        # benchmark workload (the same physics and column shape on a quarter of the columns in each
        # direction), medians over the seeds 0-4; the full workload (5 minutes of oracle setup per
        # box) is measured by --cpu-baseline-full
        ncores = os.cpu_count()
        c1 = cpu_baseline(make_box(nx=16, ny=16, nlev=8, dx=10e3, dz=1250.0, mg_levels=4), args.coarse_sweeps,
                          args.coarse_jacobi)
        nxs = 64
        cs = cpu_baseline(make_box(nx=nxs, ny=nxs, nlev=args.nlev, dx=dx, dz=dz, dt=dt, mg_levels=4),
                          args.coarse_sweeps, args.coarse_jacobi)
        scale = prob.ncell / cs["ncell"]
        cpu = {"value": cs["median_s"], "unit": "s", "cores": 1, "kind": "oracle",
               "host_cpu_count": ncores,
               "sample": (f"measured, not scaled: the oracle's FGMRES + two-level solve (condense RHS, FGMRES to 1e-8, "
                          f"recover; setup excluded) on a {nxs}x{nxs}x{args.nlev} box of the benchmark's physics and "
                          f"column shape ({cs['ncell']} cells, 1/{scale:.0f} of the benchmark's; {cs['iters']} "
                          f"iterations, as on the full box), median of seeds 0-4, 1 BLAS thread of {ncores} host cores "
                          f"(SciPy's sparse kernels are single threaded); the full box is measured by "
                          f"--cpu-baseline-full"),
               "per_cell_us": cs["median_s"] / cs["ncell"] * 1e6,
               "estimate_for_workload_s": cs["median_s"] * scale,
               "estimate_note": "the sample times the cell ratio; the oracle's time per cell grows with the mesh, so "
                                "this understates the full box",
               "measured": {"config1_box16x16x8": {"median_s": c1["median_s"], "times_s": c1["times"],
                                                   "iters": c1["iters"], "setup_s": c1["setup_s"]},
                            f"box{nxs}x{nxs}x{args.nlev}": {"median_s": cs["median_s"], "times_s": cs["times"],
                                                           "iters": cs["iters"], "setup_s": cs["setup_s"]}}}
    cpu_full = None
    if args.cpu_baseline_full or args.splu_scaling:
        cpu_full = {"host_cpu_count": os.cpu_count(), "threads": 1}
    if args.cpu_baseline_full:
        # the full box, then halved in each horizontal direction until the oracle's setup fits
        cpu_full["boxes"] = []
        nxf = args.nx
        while nxf >= 16:
            box = f"{nxf}x{nxf}x{args.nlev}"
            try:
                pf = prob if nxf == args.nx else make_box(nx=nxf, ny=nxf, nlev=args.nlev, dx=dx, dz=dz, dt=dt,
                                                          mg_levels=4)
                cf = cpu_baseline(pf, args.coarse_sweeps, args.coarse_jacobi, seeds=tuple(range(args.cpu_full_seeds)))
            except (RuntimeError, MemoryError) as err:
                cpu_full["boxes"].append({"box": box, "status": f"oracle setup failed: {str(err)[:160]}"})
                log(f"cpu baseline: {box}: oracle setup failed ({str(err)[:120]})")
                nxf //= 2
                continue
            cpu_full["boxes"].append({"box": box, "ncell": cf["ncell"], "median_s": cf["median_s"],
                                      "times_s": cf["times"], "iters": cf["iters"], "setup_s": cf["setup_s"]})
            break
    if args.splu_scaling:
        cpu_full["splu_mixed"] = splu_scaling([16, 32, 64, 128], dx, dz, dt, lambda nx: nx // 4 if nx > 16 else 8, 170)

    out = {
        "metric": "time-to-1e-8 rel residual per trace solve (s) + HBM GB/s, plain vs mixed/learned",
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"periodic box {args.nx}x{args.nx}x{args.nlev}, dx=5km, dz=250m, dt=600s, "
                               f"RT0/Q0/trace, FGMRES(30)+two-level (1 pre/2 post, 4-level V-cycle, coarsest "
                               f"{coarsest_desc(args)}), rtol 1e-8",
                   "ncell": ncell, "ntrace": ntr},
        "solves_per_s": 1.0 / sec,
        "iters": its,
        "rel_res": max(i["rel_res"] for i in infos),
        "setup_s": setup_s,
        "hbm_gbs_algorithmic": per_solve_bytes / sec / 1e9,
        "hbm_frac_algorithmic": per_solve_bytes / sec / 1e9 / PEAK_HBM_GBS,
        "bytes_per_solve": per_solve_bytes,
        "bytes_per_solve_note": "every launch of this implementation counted by what its definition reads and writes once",
        "hbm_gbs_model": model_bytes / sec / 1e9,
        "hbm_frac_model": model_bytes / sec / 1e9 / PEAK_HBM_GBS,
        "bytes_per_solve_model": model_bytes,
        "bytes_per_solve_model_note": ("what the method must move per solve, independent of how it is split into "
                                       "launches: 1.0 KB + 2.01 KB m + 24 m (m + 1) + 24 (m + 1) B per cell "
                                       "for m iterations"),
        "sec_per_solve_with_dominant_kernel_events": sec_dom,
        "roofline": {"bound": "hbm", "kernel": "k_rows<double,double,double,OP_SMOOTH>", "achieved": ls_gbs,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ls_gbs / PEAK_HBM_GBS, "traffic": measured_traffic(args.nx, args.nlev),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1, copy-calibrated)",
                     "launches": ls_launches, "avg_ms": ls_avg_ms, "bytes_per_launch": ls_bytes},
        "kernel_ms": {k: {"launches": v[0], "total_ms": v[1]} for k, v in fams.items()},
        "kernel_ms_note": "from a third run of the same solves with events around every family",
        "mixed": mixed,
        "learned": learned_out,
        "configurations": configs_out,
        "appendix_b": appb_out,
        "sphere": sphere_out,
        "c384": c384_out,
        "p1": p1_out,
        "cpu_baseline": cpu,
        "cpu_baseline_full": cpu_full,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
