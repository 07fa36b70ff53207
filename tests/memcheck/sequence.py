"""Drive the C ABI of a library built by build.py through the call sequences that matter for memory
safety, on small synthetic boxes (run under AddressSanitizer by tests/test_memcheck.py).

The sequences cover: setup, condensation, every trace-space operator, FGMRES in both precisions
(with restarts), recovery, profiling, the learned stage (a training step as the first network call
of a context, batch sizes that grow and shrink, the solve with the stage in both precisions, the
non-finite fallback) and argument errors.  A few results are checked for sanity (the solve meets
its tolerance, the network output matches the oracle's formula); the parity tests proper run on the
GPU.
"""

from __future__ import annotations

import ctypes
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import nn as onn  # noqa: E402
from paper_2210_11797_amd import _native as N  # noqa: E402
from paper_2210_11797_amd import learned  # noqa: E402
from oracle.problem import OracleProblem, cells_from_soa  # noqa: E402
from synth import make_box, make_rhs, make_rhs_sphere, make_sphere  # noqa: E402

vp = ctypes.c_void_p


def P(a):
    return a.ctypes.data_as(vp)


class Ctx:
    def __init__(self, lib, prob, order=0, **kw):
        self.lib, self.prob, self.order = lib, prob, order
        keep = []
        levels = N.levels_of(prob)
        lv = (N._Level * len(levels))()
        for i, L in enumerate(levels):
            arr = {}
            for key in ("col_edge", "edge_col", "edge_lf"):
                a = np.ascontiguousarray(L[key], np.int32)
                keep.append(a)
                arr[key] = a.ctypes.data_as(N._i32p)
            par = None
            if L["parent"] is not None:
                a = np.ascontiguousarray(L["parent"], np.int32)
                keep.append(a)
                par = a.ctypes.data_as(N._i32p)
            lv[i] = N._Level(int(L["ncol"]), arr["col_edge"], arr["edge_col"], arr["edge_lf"], par)
        dz = np.ascontiguousarray(prob.dz, np.float64)
        self.shell = getattr(prob, "geom", "box") == "shell"
        geom, cptr, rptr = N.GEOM_BOX, None, None
        if self.shell:
            ch = np.ascontiguousarray(prob.corners, np.float64)
            rh = np.ascontiguousarray(prob.radius, np.float64)
            keep += [ch, rh]
            geom, cptr, rptr = N.GEOM_SHELL, ch.ctypes.data_as(N._f64p), rh.ctypes.data_as(N._f64p)
        self._keep = keep
        mesh = N._Mesh(prob.nlev, len(levels), lv, prob.dx, prob.dy, dz.ctypes.data_as(N._f64p), order, geom, cptr,
                       rptr)
        base = dict(dt=prob.dt, tau_u=prob.tau_u, tau_rho=prob.tau_rho, tau_theta=prob.tau_theta, cp=prob.cp,
                    rd=prob.rd)
        base.update(kw)
        self.params = N.Params(**base)
        cp = self.params.to_c()
        self.h = vp()
        rc = lib.hyb_create(ctypes.byref(mesh), ctypes.byref(cp), None, ctypes.byref(self.h))
        assert rc == 0, rc
        nt, nc = ctypes.c_int64(), ctypes.c_int64()
        lib.hyb_sizes(self.h, ctypes.byref(nt), ctypes.byref(nc), None)
        self.ntrace, self.ncell = nt.value, nc.value
        f = lambda a: np.ascontiguousarray(a, np.float64)  # noqa: E731
        self.call("hyb_assemble_local", P(f(prob.theta_w)), P(f(prob.exner_hat_w)), P(f(prob.exner_c)),
                  P(f(prob.rho_c)))
        self.call("hyb_condense", None, None, None)

    def call(self, name, *args):
        rc = getattr(self.lib, name)(self.h, *args)
        if rc < 0:
            raise RuntimeError(f"{name} failed ({rc}): {self.lib.hyb_last_error(self.h).decode()}")
        return rc

    def set(self, **kw):
        for k, v in kw.items():
            setattr(self.params, k, v)
        cp = self.params.to_c()
        self.call("hyb_set_params", ctypes.byref(cp))

    def rhs(self, seed):
        r_ub, r_pi = make_rhs_sphere(self.prob, seed) if self.shell else make_rhs(self.prob, seed)
        r_ub, r_pi = np.ascontiguousarray(r_ub, np.float64), np.ascontiguousarray(r_pi, np.float64)
        b = np.empty(self.ntrace)
        self.call("hyb_condense", P(r_ub), P(r_pi), P(b))
        return r_ub, r_pi, b

    def solve(self, b, rtol, maxit=500):
        lam = np.zeros(self.ntrace)
        hist = (ctypes.c_double * 64)()
        info = N._Info(0, 0, 0, 0.0, ctypes.cast(hist, N._f64p), 64, 0)
        rc = self.call("hyb_solve", P(b), P(lam), rtol, maxit, ctypes.byref(info))
        return rc, info, lam

    def residual(self, b, lam):
        y = np.empty(self.ntrace)
        self.call("hyb_trace_apply", P(lam), P(y))
        return np.linalg.norm(b - y) / np.linalg.norm(b)

    def close(self):
        self.lib.hyb_destroy(self.h)


def check(cond, what):
    print(("ok   " if cond else "FAIL ") + what, flush=True)
    if not cond:
        sys.exit(3)


def solver_sequence(lib):
    prob = make_box(nx=8, ny=6, nlev=7, dx=5e3, dz=250.0, mg_levels=2, perturb=0.05, seed=4)
    c = Ctx(lib, prob, restart=5)
    r_ub, r_pi, b = c.rhs(1)
    y, z, cells = np.empty(c.ntrace), np.empty(c.ntrace), np.empty(c.ncell)
    c.call("hyb_trace_apply", P(b), P(y))
    c.call("hyb_precondition", P(b), P(z))
    c.call("hyb_restrict", P(b), P(cells), 0)
    c.call("hyb_restrict", P(b), P(cells), 1)
    rc, info, lam = c.solve(b, 1e-10)
    check(rc == 0 and info.restarts > 0 and c.residual(b, lam) <= 1.01e-10,
          f"fp64 FGMRES(5): {info.iters} iterations, {info.restarts} restarts")
    u_b, pi = np.empty(6 * c.ncell), np.empty(c.ncell)
    c.call("hyb_recover", P(r_ub), P(r_pi), P(lam), P(u_b), P(pi))
    c.set(coarse_mode=1, n_pre=2, n_post=1)  # LineSmooth alone (single-level configuration)
    c.call("hyb_precondition", P(b), P(z))
    rc, info, lam = c.solve(b, 1e-8, maxit=2000)
    check(rc == 0 and c.residual(b, lam) <= 1.01e-8, f"single-level FGMRES(5): {info.iters} iterations")
    c.set(coarse_mode=0, n_pre=1, n_post=2)
    # the Krylov coarse solve (BiCGStab + V-cycle on the coarse pressure system): loose and tight
    for crt in (1e-2, 1e-14):
        c.set(coarse_mode=2, coarse_rtol=crt)
        c.call("hyb_precondition", P(b), P(z))
        rc, info, lam = c.solve(b, 1e-8)
        check(rc == 0 and c.residual(b, lam) <= 1.01e-8, f"Krylov coarse solve to {crt:.0e}: {info.iters} iterations")
    bad = N.Params(**{**c.params.__dict__, "precision": N.PREC_MIXED})
    cp_bad = bad.to_c()
    check(lib.hyb_set_params(c.h, ctypes.byref(cp_bad)) < 0, "the Krylov coarse solve in the mixed form is rejected")
    c.set(coarse_mode=0)
    c.set(precision=N.PREC_MIXED, restart=30)
    c.call("hyb_precondition", P(b), P(z))
    rc, info, lam = c.solve(b, 1e-8)
    check(rc == 0 and c.residual(b, lam) <= 1.01e-8, f"mixed FGMRES: {info.iters} iterations")
    # LineSmooth with the column matrices cached per 2x2 patch (the parent coarse column), against
    # the oracle's variant, in both precisions
    # (100 eps cond(H) as in the parity tests; the variant moves z by ~4e-7 on this machine)
    orc = OracleProblem(prob, with_mixed=False, smoother_patch=True)
    c.set(precision=N.PREC_FP64, restart=30, smoother_patch=1)
    c.call("hyb_precondition", P(b), P(z))
    zref = orc.pc(b)
    ez = float(np.abs(z - zref).max() / np.abs(zref).max())
    moved = float(np.abs(OracleProblem(prob, with_mixed=False).pc(b) - zref).max() / np.abs(zref).max())
    rc, info, lam = c.solve(b, 1e-10)
    check(ez <= 1.5e-9 and moved > 100 * ez and rc == 0 and c.residual(b, lam) <= 1.01e-10,
          f"patch-cached LineSmooth: preconditioner vs oracle {ez:.1e} (variant moves it {moved:.1e}), "
          f"FGMRES {info.iters} iterations")
    c.set(precision=N.PREC_MIXED)
    rc, info, lam = c.solve(b, 1e-8)
    check(rc == 0 and c.residual(b, lam) <= 1.01e-8, f"patch-cached LineSmooth, mixed: {info.iters} iterations")
    # failure injection: Gamma = 0 leaves the cycle its LineSmooth sweeps (bitwise the smoother-only
    # configuration with the same sweeps), and unknown debug bits are rejected
    c.set(precision=N.PREC_FP64, smoother_patch=0, debug=N.HYB_DEBUG_ZERO_GAMMA)
    z0 = np.empty(c.ntrace)
    c.call("hyb_precondition", P(b), P(z0))
    c.set(debug=0, coarse_mode=1)
    z1 = np.empty(c.ntrace)
    c.call("hyb_precondition", P(b), P(z1))
    c.set(coarse_mode=0)
    bad = N.Params(**{**c.params.__dict__, "debug": 8})
    cp_bad = bad.to_c()
    check(np.array_equal(z0, z1) and lib.hyb_set_params(c.h, ctypes.byref(cp_bad)) < 0,
          "Gamma = 0 gives the smoother-only cycle bit for bit; unknown debug bits rejected")
    # the restriction reading child pairs as vectors and through the children map: same bits
    for prec in (N.PREC_FP64, N.PREC_MIXED):
        zz = []
        for flag in (0, N.HYB_DEBUG_UNPAIRED_RESTRICT):
            c.set(precision=prec, debug=flag)
            zq = np.empty(c.ntrace)
            c.call("hyb_precondition", P(b), P(zq))
            rc, info, lam = c.solve(b, 1e-8)
            zz.append((zq, info.iters, lam))
        c.set(debug=0)
        check(np.array_equal(zz[0][0], zz[1][0]) and zz[0][1] == zz[1][1] and np.array_equal(zz[0][2], zz[1][2]),
              f"paired and unpaired restriction agree bit for bit (precision {prec}, {zz[0][1]} iterations)")
    c.set(precision=N.PREC_MIXED)
    c.call("hyb_profile", 1)
    c.solve(b, 1e-6)
    n, ms = ctypes.c_int64(), ctypes.c_double()
    for fam in ("smooth_rows", "smooth_rows0", "thomas", "trace_apply", "mg_smooth", "restrict", "prolong",
                "krylov", "cell_solve", "nn"):
        c.call("hyb_profile_read", fam.encode(), ctypes.byref(n), ctypes.byref(ms))
    c.call("hyb_profile", 0)
    c.call("hyb_profile_family", b"krylov")
    c.solve(b, 1e-6)
    c.call("hyb_profile_read", b"krylov", ctypes.byref(n), ctypes.byref(ms))
    check(n.value > 0 and lib.hyb_profile_read(c.h, b"smooth_rows", ctypes.byref(n), ctypes.byref(ms)) == 0
          and n.value == 0, "single-family profiling records that family only")
    check(lib.hyb_profile_family(c.h, b"nonsense") < 0, "unknown profiling family rejected")
    c.call("hyb_profile", 0)
    # restart cycles longer than the delayed-reorthogonalisation limit take the three-pass and
    # the conditional second-pass Gram-Schmidt paths
    c.set(precision=N.PREC_FP64, restart=40)
    rc, info, lam = c.solve(b, 0.0, maxit=36)
    res = c.residual(b, lam)
    check(info.iters == 36 and res <= 1e-12, f"fp64 FGMRES(40), 36 steps without a tolerance: residual {res:.1e}")
    c.set(restart=30)
    rc, info, lam = c.solve(b, 1e-20, maxit=3000)
    check(rc == N.HYB_STAGNATED and info.iters < 3000 and c.residual(b, lam) <= 1e-13,
          f"a tolerance below the rounding floor ends as stagnated after {info.iters} iterations")
    # the allocation-free solve (static reduction scratch) gives hyb_solve's iterate, also on a
    # second, smaller context after it
    for prec in (N.PREC_FP64, N.PREC_MIXED):
        c.set(precision=prec)
        rc, info, lam = c.solve(b, 1e-9)
        lam_na = np.zeros(c.ntrace)
        info_na = N._Info(0, 0, 0, 0.0, None, 0, 0)
        rc_na = c.call("hyb_solve_noalloc", P(b), P(lam_na), 1e-9, 500, ctypes.byref(info_na))
        check(rc_na == 0 and info_na.iters == info.iters and np.array_equal(lam, lam_na),
              f"hyb_solve_noalloc = hyb_solve (precision {prec}, {info.iters} iterations)")
    c.set(precision=N.PREC_FP64)
    cs = Ctx(lib, make_box(nx=3, ny=2, nlev=2, dx=5e3, dz=250.0, mg_levels=1, seed=9))
    _, _, bs = cs.rhs(1)
    rc, info, lam = cs.solve(bs, 1e-10)
    lam_na = np.zeros(cs.ntrace)
    rc_na = cs.call("hyb_solve_noalloc", P(bs), P(lam_na), 1e-10, 500, None)
    check(rc_na == 0 and np.array_equal(lam, lam_na), "hyb_solve_noalloc on a smaller second context")
    cs.set(restart=62)
    check(lib.hyb_solve_noalloc(cs.h, P(bs), P(lam_na), 1e-10, 500, None) < 0,
          "hyb_solve_noalloc rejects a restart whose partials exceed the static scratch")
    cs.close()
    c2 = Ctx(lib, make_box(nx=4, ny=4, nlev=66, dx=5e3, dz=150.0, mg_levels=2, seed=8))  # nlev > 64: Thomas path
    _, _, b2 = c2.rhs(3)
    rc2, info2, lam2 = c2.solve(b2, 1e-10)
    check(rc2 == 0 and c2.residual(b2, lam2) <= 1.01e-10, f"66 levels (two-kernel smoother): {info2.iters} iterations")
    c2.close()
    # argument errors come back as codes
    check(lib.hyb_restrict(c.h, P(b), P(cells), 4) < 0 and lib.hyb_restrict(c.h, P(b), P(cells), -1) < 0,
          "bad restriction modes rejected")
    check(lib.hyb_solve(c.h, P(b), P(b), 1e-8, 10, None) < 0, "aliased solve vectors rejected")
    c.close()


def network_sequence(lib):
    prob = make_box(nx=8, ny=6, nlev=7, dx=5e3, dz=250.0, mg_levels=2, perturb=0.05, seed=5)
    c = Ctx(lib, prob)
    nc = c.ncell
    rng = np.random.default_rng(0)
    check(lib.hyb_nn_forward(c.h, None, None, 1) < 0, "network call before weights rejected")
    w = learned.init_params(16, seed=2)
    c.call("hyb_nn_set_weights", P(w), w.size)
    # the preconditioner with the stage before any solve (Krylov scratch not yet allocated)
    v, z = rng.standard_normal(c.ntrace), np.empty(c.ntrace)
    for prec in (N.PREC_MIXED, N.PREC_FP64):
        c.set(learned=1, precision=prec)
        c.call("hyb_precondition", P(v), P(z))
    cells = np.empty(nc)
    c.call("hyb_restrict", P(v), P(cells), 2)
    c.call("hyb_restrict", P(v), P(cells), 3)
    c.set(learned=0)
    # energy loss: first with a batch of 2, then a larger one (buffers grow)
    for ns in (2, 4):
        xe = rng.standard_normal((ns, nc)).astype(np.float32)
        re = rng.standard_normal((ns, nc))
        el = ctypes.c_double()
        ge = np.empty(w.size, np.float32)
        c.call("hyb_nn_energy_grad", P(xe), P(re), ns, ctypes.byref(el), P(ge))
        c.call("hyb_nn_energy_train_step", P(xe), P(re), ns, ctypes.c_float(1e-3), None)
    check(np.isfinite(el.value) and np.all(np.isfinite(ge)), f"energy loss and gradient: {el.value:.3e}")
    # training pairs in the library: the cycle step, residual update and normalisation against the
    # same steps through the separate calls; a gathered step against the step on the copied batch
    _, _, bp = c.rhs(4)
    r_lib, r_ref = bp.copy(), bp.copy()
    xp, rp = np.empty((2, nc), np.float32), np.empty((2, nc))
    zz, sz, gc, pt = np.empty(c.ntrace), np.empty(c.ntrace), np.empty(nc), np.empty(nc)
    ok = True
    for k in range(2):
        sc = ctypes.c_double()
        c.call("hyb_nn_cycle_pair", P(r_lib), P(xp[k]), P(rp[k]), ctypes.byref(sc))
        c.call("hyb_precondition", P(r_ref), P(zz))
        c.call("hyb_trace_apply", P(zz), P(sz))
        r_ref -= sz
        c.call("hyb_restrict", P(r_ref), P(gc), 0)
        c.call("hyb_restrict", P(r_ref), P(pt), 3)
        s_ref = np.sqrt(np.mean(gc * gc))
        ok &= abs(sc.value - s_ref) <= 1e-12 * s_ref and np.abs(r_lib - r_ref).max() <= 1e-12 * np.abs(r_ref).max()
        ok &= np.abs(xp[k] - (gc / s_ref).astype(np.float32)).max() <= 1e-6 * np.abs(xp[k]).max()
        ok &= np.abs(rp[k] - pt / s_ref).max() <= 1e-12 * np.abs(rp[k]).max()
    check(ok, "hyb_nn_cycle_pair = precondition, S z, residual, Gamma P^T r / s and P^T r / s")
    zero, xz, rz = np.zeros(c.ntrace), np.empty(nc, np.float32), np.empty(nc)
    check(c.call("hyb_nn_cycle_pair", P(zero), P(xz), P(rz), None) == N.HYB_BREAKDOWN,
          "a vanished residual gives HYB_BREAKDOWN")
    c.call("hyb_nn_set_weights", P(w), w.size)
    idx = np.array([1, 0, 1], np.int32)
    l1, l2 = ctypes.c_double(), ctypes.c_double()
    c.call("hyb_nn_energy_train_step_pairs", P(xp), P(rp), 2, P(idx), 3, ctypes.c_float(1e-3), ctypes.byref(l1))
    w1 = np.empty(w.size, np.float32)
    c.call("hyb_nn_get_weights", P(w1), w1.size)
    c.call("hyb_nn_set_weights", P(w), w.size)
    xg, rg = np.ascontiguousarray(xp[idx]), np.ascontiguousarray(rp[idx])
    c.call("hyb_nn_energy_train_step", P(xg), P(rg), 3, ctypes.c_float(1e-3), ctypes.byref(l2))
    w2 = np.empty(w.size, np.float32)
    c.call("hyb_nn_get_weights", P(w2), w2.size)
    bad_idx = np.array([2], np.int32)
    check(l1.value == l2.value and np.array_equal(w1, w2)
          and lib.hyb_nn_energy_train_step_pairs(c.h, P(xp), P(rp), 2, P(bad_idx), 1, ctypes.c_float(1e-3), None) < 0,
          "gathered training step = step on the copied batch; an index out of range is rejected")
    # resuming from the Adam state: 2 + 2 steps with the state carried over = 4 steps in a row
    def steps(k):
        for _ in range(k):
            c.call("hyb_nn_energy_train_step", P(xg), P(rg), 3, ctypes.c_float(1e-3), None)
    c.call("hyb_nn_set_weights", P(w), w.size)
    steps(4)
    w4 = np.empty(w.size, np.float32)
    c.call("hyb_nn_get_weights", P(w4), w4.size)
    c.call("hyb_nn_set_weights", P(w), w.size)
    steps(2)
    w2s, am, av, ast = np.empty(w.size, np.float32), np.empty(w.size, np.float32), np.empty(w.size, np.float32), \
        ctypes.c_int64()
    c.call("hyb_nn_get_weights", P(w2s), w2s.size)
    c.call("hyb_nn_get_state", P(am), P(av), w.size, ctypes.byref(ast))
    c.call("hyb_nn_set_weights", P(w), w.size)  # resets the state
    c.call("hyb_nn_set_weights", P(w2s), w2s.size)
    c.call("hyb_nn_set_state", P(am), P(av), w.size, ast.value)
    steps(2)
    w22 = np.empty(w.size, np.float32)
    c.call("hyb_nn_get_weights", P(w22), w22.size)
    neg = -np.abs(av) - 1.0
    check(ast.value == 2 and np.array_equal(w4, w22) and lib.hyb_nn_set_state(c.h, P(am), P(neg), w.size, 2) < 0,
          "training resumed from the Adam state = training without a break; a negative moment is rejected")
    for fp32 in (1, 0):  # the FP32 reference passes and the BF16 matrix-core ones
        c.set(nn_fp32=fp32)
        c.call("hyb_nn_set_weights", P(w), w.size)
        loss = ctypes.c_float()
        # a training step as the very first network call (activation buffers not yet allocated)
        x3 = rng.standard_normal((3, nc)).astype(np.float32)
        t3 = rng.standard_normal((3, nc)).astype(np.float32)
        c.call("hyb_nn_train_step", P(x3), P(t3), 3, ctypes.c_float(1e-3), ctypes.byref(loss))
        check(np.isfinite(loss.value), f"first call is a training step (batch 3, fp32 {fp32}): loss {loss.value:.4f}")
        g = np.empty(w.size, np.float32)
        c.call("hyb_nn_loss_grad", P(x3[:2].copy()), P(t3[:2].copy()), 2, ctypes.byref(loss), P(g))
        x5 = rng.standard_normal((5, nc)).astype(np.float32)  # larger batch: buffers grow
        y5 = np.empty((5, nc), np.float32)
        c.call("hyb_nn_forward", P(x5), P(y5), 5)
        c.call("hyb_nn_train_step", P(x5), P(x5), 5, ctypes.c_float(1e-3), None)
        x1 = x5[:1].copy()
        y1 = np.empty((1, nc), np.float32)
        c.call("hyb_nn_forward", P(x1), P(y1), 1)
        wc = np.empty(w.size, np.float32)
        c.call("hyb_nn_get_weights", P(wc), wc.size)
        W, bias = learned.unpack(wc)
        st = onn.static_inputs(prob.dx * prob.dy * np.repeat(np.diff(prob.z), prob.ncol), prob.z, prob.ncol)
        ref = onn.forward(x1[0].astype(np.float64), [onn.bf16_round(a) for a in W], bias,
                          onn.neighbour_table(prob.nx, prob.ny), prob.nlev, static=st)[0]
        err = float(np.abs(y1[0] - ref).max() / np.abs(ref).max())
        check(err <= (1e-5 if fp32 else 2.0**-6),
              f"forward after training matches the oracle's formula (fp32 {fp32}): {err:.1e}")
    _, _, b = c.rhs(2)
    for prec in (N.PREC_FP64, N.PREC_MIXED):
        c.set(learned=1, precision=prec)
        rc, info, lam = c.solve(b, 1e-8, maxit=40)
        check(rc >= 0, f"solve with the learned stage (precision {prec}): {info.iters} iterations")
    wo = w.copy()
    wo[: 16 * learned.NIN * 45] = np.repeat(np.where(np.arange(16) % 2 == 0, 1e30, -1e30), learned.NIN * 45)
    wo[16 * learned.NIN * 45 + 16: 16 * learned.NIN * 45 + 16 + 16 * 16 * 45] = 1e30
    c.call("hyb_nn_set_weights", P(wo), wo.size)
    c.set(precision=N.PREC_FP64)
    rc, info, lam = c.solve(b, 1e-8)
    check(rc == 0 and info.fallbacks == info.iters, f"overflowing network falls back: {info.fallbacks}/{info.iters}")
    c.call("hyb_nn_set_weights", P(w), w.size)
    c.set(debug=N.HYB_DEBUG_NAN_STAGE)
    rc, info, lam = c.solve(b, 1e-8)
    c.set(debug=0, learned=0)
    check(rc == 0 and info.fallbacks == info.iters, f"a NaN network output falls back: {info.fallbacks}/{info.iters}")
    c.close()


def p1_sequence(lib):
    """Order 1: assembly, condensation, S x, B_lambda and recovery against the oracle's p = 1 system
    (a sanity check of the same code the GPU runs)."""
    from oracle import p1 as op1
    from oracle.mesh import BoxMesh

    prob = make_box(nx=3, ny=2, nlev=3, dx=5e3, dz=250.0, mg_levels=1, perturb=0.05, seed=6)
    c = Ctx(lib, prob, order=1)
    mesh = BoxMesh(prob.nx, prob.ny, prob.nlev, prob.dx, prob.dy, prob.z)
    h = op1.HybridP1(mesh, op1.local_matrices(mesh, prob))
    check(c.ntrace == h.ntrace, f"order 1: {c.ntrace} trace unknowns")
    rng = np.random.default_rng(7)
    x = rng.standard_normal(c.ntrace)
    y = np.empty(c.ntrace)
    c.call("hyb_trace_apply", P(x), P(y))
    ref = h.S @ x
    check(np.abs(y - ref).max() <= 1e-11 * np.abs(ref).max(), "order 1: S x matches the oracle")
    r_u = rng.standard_normal((36, c.ncell))
    r_p = rng.standard_normal((8, c.ncell))
    b = np.empty(c.ntrace)
    c.call("hyb_condense", P(r_u), P(r_p), P(b))
    bref = h.rhs(r_u.T.copy(), r_p.T.copy())
    check(np.abs(b - bref).max() <= 1e-11 * np.abs(bref).max(), "order 1: B_lambda matches the oracle")
    u, pi = np.empty((36, c.ncell)), np.empty((8, c.ncell))
    c.call("hyb_recover", P(r_u), P(r_p), P(x), P(u), P(pi))
    uref, pref = h.recover(x, r_u.T.copy(), r_p.T.copy())
    check(np.abs(u.T - uref).max() <= 1e-10 * np.abs(uref).max() and np.abs(pi.T - pref).max() <= 1e-10 * np.abs(pref).max(),
          "order 1: recovery matches the oracle")
    # the two-level preconditioner and the solve against the oracle's
    from oracle.problem import OracleProblem

    tl = op1.TwoLevelP1(mesh, h.S, OracleProblem(prob).H, mg_levels=1)
    z = np.empty(c.ntrace)
    c.call("hyb_precondition", P(b), P(z))
    zref = tl(b)
    check(np.abs(z - zref).max() <= 1e-9 * np.abs(zref).max(), "order 1: preconditioner matches the oracle")
    rc, info, lam = c.solve(b, 1e-12)
    lref = op1.spla.splu(h.S.tocsc()).solve(b)
    check(rc == 0 and np.abs(lam - lref).max() <= 1e-9 * np.abs(lref).max(),
          f"order 1: FGMRES solve matches the direct solution ({info.iters} iterations)")
    cells = np.empty(c.ncell)
    check(lib.hyb_restrict(c.h, P(b), P(cells), 0) < 0, "order 1: calls it does not provide are rejected")
    c.close()
    # the mixed form: FP64 outer operator, FP32 copy of S_K inside the preconditioner
    cx = Ctx(lib, prob, order=1, precision=N.PREC_MIXED)
    zx = np.empty(cx.ntrace)
    cx.call("hyb_precondition", P(b), P(zx))
    ez = np.abs(zx - z).max() / np.abs(z).max()
    rc, info, lam_x = cx.solve(b, 1e-10)
    check(0 < ez <= 1e-5 and rc == 0 and cx.residual(b, lam_x) <= 1.01e-10,
          f"order 1, mixed form: preconditioner vs FP64 {ez:.1e}, FGMRES {info.iters} iterations")
    cx.close()
    # S_K condensed on matrix cores (FP32, and BF16 split into hi + lo) against the FP64 operator
    for prec, tol in ((N.PREC_MFMA_FP32, 1e-5), (N.PREC_MFMA_BF16X, 1e-4)):
        cm = Ctx(lib, prob, order=1, precision=prec)
        ym = np.empty(cm.ntrace)
        cm.call("hyb_trace_apply", P(x), P(ym))
        err = np.abs(ym - ref).max() / np.abs(ref).max()
        check(err <= tol, f"order 1, condensation mode {prec}: S x error vs FP64 {err:.1e}")
        rc, info, lam_m = cm.solve(b, 1e-8)
        check(rc == 0 and cm.residual(b, lam_m) <= 1.01e-8,
              f"order 1, condensation mode {prec}: FGMRES on the FP32 S_K ({info.iters} iterations)")
        # a change of arithmetic asks for the condensation again, and FP64 restores the exact operator
        cm.set(precision=N.PREC_FP64)
        check(lib.hyb_trace_apply(cm.h, P(x), P(ym)) < 0, "order 1: a new precision rejects S x until condensed")
        cm.call("hyb_condense", None, None, None)
        cm.call("hyb_trace_apply", P(x), P(ym))
        check(np.abs(ym - ref).max() <= 1e-11 * np.abs(ref).max(), "order 1: FP64 condensation after a switch")
        cm.close()


def sphere_sequence(lib):
    # the extruded cubed sphere with rotation: shell assembly (twice: without and with the Coriolis
    # term), condensation, S x, B_lambda, the preconditioner, FGMRES in both precisions, recovery;
    # S x and the recovery against the oracle
    prob = make_sphere(4, 5, mg_levels=2, perturb=0.05, seed=3)
    # a column frame turned the wrong way (corners 1 and 2 swapped) is rejected at create
    bad = make_sphere(4, 5, mg_levels=2, seed=3)
    bad.corners = np.ascontiguousarray(bad.corners.copy())
    bad.corners[[1, 2], :, 7] = bad.corners[[2, 1], :, 7]
    try:
        Ctx(lib, bad, omega_rot=bad.omega_rot)
        rejected = False
    except AssertionError:
        rejected = True
    check(rejected, "sphere: a left-handed column frame is rejected")
    c = Ctx(lib, prob, omega_rot=prob.omega_rot)
    o = OracleProblem(prob)
    r_ub, r_pi, b = c.rhs(2)
    ruc, rpc = cells_from_soa(r_ub, r_pi)
    bref = o.hyb.rhs(ruc, rpc)
    check(np.abs(b - bref).max() <= 1e-11 * np.abs(bref).max(), "sphere: B_lambda against the oracle")
    x = np.random.default_rng(0).standard_normal(c.ntrace)
    y, z = np.empty(c.ntrace), np.empty(c.ntrace)
    c.call("hyb_trace_apply", P(x), P(y))
    ref = o.hyb.S @ x
    check(np.abs(y - ref).max() <= 1e-11 * np.abs(ref).max(), "sphere: S x against the oracle")
    c.call("hyb_precondition", P(b), P(z))
    zref = o.pc(b)
    check(np.abs(z - zref).max() <= 1e-9 * np.abs(zref).max(),
          "sphere: preconditioner (lumped mass without the Coriolis term) against the oracle")
    # the theta' / rho' elimination and back-substitution against the oracle (in place too)
    from oracle.elimination import back_substitute, eliminate_rhs
    from oracle.local import shell_cells, shell_fields, shell_map

    rng = np.random.default_rng(6)
    L, ncol = prob.nlev, prob.ncol
    e_ub, e_rho, e_th, e_pi = (rng.standard_normal((6, L, ncol)), rng.standard_normal((L, ncol)),
                               rng.standard_normal((L + 1, ncol)), rng.standard_normal((L, ncol)))
    ub_bar, pi_bar = e_ub.copy(), e_pi.copy()
    c.call("hyb_eliminate", P(ub_bar), P(e_rho), P(e_th), P(pi_bar), P(ub_bar), P(pi_bar))
    tm = o.mesh
    U, r0, r1 = shell_cells(tm, prob)
    cm, fl = shell_map(U, r0, r1), shell_fields(tm, prob)
    cs = dict(dt=prob.dt, tau_u=prob.tau_u, tau_rho=prob.tau_rho, tau_theta=prob.tau_theta, cp=prob.cp)
    kk, cc = tm.cell_layer, tm.cell_col
    rb, rp = eliminate_rhs(cm, True, fl, cs, e_ub.reshape(6, -1).T, e_rho.ravel(), e_th[kk, cc], e_th[kk + 1, cc],
                           e_pi.ravel())
    rho_e, th_e = np.empty((L, ncol)), np.empty((2, L, ncol))
    c.call("hyb_back_substitute", P(e_rho), P(e_th), P(e_ub), P(rho_e), P(th_e))
    rho_r, th_r = back_substitute(cm, True, fl, cs, e_rho.ravel(), e_th[kk, cc], e_th[kk + 1, cc], e_ub.reshape(6, -1).T)
    check(np.abs(ub_bar.reshape(6, -1).T - rb).max() <= 1e-12 * np.abs(rb).max()
          and np.abs(pi_bar.ravel() - rp).max() <= 1e-12 * np.abs(rp).max()
          and np.abs(rho_e.ravel() - rho_r).max() <= 1e-12 * np.abs(rho_r).max()
          and np.abs(th_e.reshape(2, -1).T - th_r).max() <= 1e-12 * np.abs(th_r).max(),
          "sphere: theta' / rho' elimination and back-substitution against the oracle")
    check(lib.hyb_back_substitute(c.h, P(e_rho), P(e_th), P(e_ub), P(e_ub), P(th_e)) < 0,
          "back-substitution outputs aliasing an input rejected")
    rc, info, lam = c.solve(b, 1e-10)
    check(rc == 0 and c.residual(b, lam) <= 1.01e-10, f"sphere: fp64 FGMRES {info.iters} iterations")
    u_b, pi = np.empty(6 * c.ncell), np.empty(c.ncell)
    c.call("hyb_recover", P(r_ub), P(r_pi), P(lam), P(u_b), P(pi))
    _, pref = o.hyb.recover(lam, ruc, rpc)
    check(np.abs(pi - pref).max() <= 1e-9 * np.abs(pref).max(), "sphere: recovery against the oracle")
    c.set(precision=N.PREC_MIXED)
    rc, info, lam = c.solve(b, 1e-8)
    check(rc == 0 and c.residual(b, lam) <= 1.01e-8, f"sphere: mixed FGMRES {info.iters} iterations")
    # the network on the frame-following neighbourhood (zero padded at the cube vertices): forward
    # and gradients against the oracle, a training step, the solve with the stage
    rng = np.random.default_rng(1)
    w = learned.init_params(16, seed=3)
    w[16 * learned.NIN * 45 : 16 * learned.NIN * 45 + 16] = rng.standard_normal(16) * 0.1
    c.call("hyb_nn_set_weights", P(w), w.size)
    nb = onn.neighbour_table_from_tables(prob.col_edge, prob.edge_col, prob.edge_lf)
    W, bias = learned.unpack(w)
    Wr = [onn.bf16_round(a) for a in W]
    x2 = rng.standard_normal((2, c.ncell)).astype(np.float32)
    t2 = rng.standard_normal((2, c.ncell)).astype(np.float32)
    st = onn.static_inputs(o.loc["m3"], prob.z, prob.ncol)
    yref = np.stack([onn.forward(x2[i].astype(np.float64), Wr, bias, nb, prob.nlev, static=st)[0] for i in range(2)])
    refs = [onn.loss_and_grads(x2[i].astype(np.float64), t2[i].astype(np.float64), Wr, bias, nb, prob.nlev, static=st)
            for i in range(2)]
    gref = learned.pack([0.5 * (refs[0][1][j] + refs[1][1][j]) for j in range(3)],
                        [0.5 * (refs[0][2][j] + refs[1][2][j]) for j in range(3)]).astype(np.float64)
    # the FP32 reference passes to the oracle's tolerances, the BF16 matrix-core ones within 2^-6
    for fp32, tol_y, tol_g in ((1, 1e-5, 1e-4), (0, 2.0**-6, 2.0**-5)):
        c.set(nn_fp32=fp32)
        y2 = np.empty((2, c.ncell), np.float32)
        c.call("hyb_nn_forward", P(x2), P(y2), 2)
        check(np.abs(y2 - yref).max() <= tol_y * np.abs(yref).max(),
              f"sphere: network forward against the oracle (fp32 {fp32})")
        loss, g = ctypes.c_float(), np.empty(w.size, np.float32)
        c.call("hyb_nn_loss_grad", P(x2), P(t2), 2, ctypes.byref(loss), P(g))
        gerr = np.abs(g - gref).max() / np.abs(gref).max()
        check(gerr <= tol_g, f"sphere: network gradients against the oracle (fp32 {fp32}: {gerr:.1e})")
    c.call("hyb_nn_train_step", P(x2), P(t2), 2, ctypes.c_float(1e-3), None)
    c.set(learned=1, precision=N.PREC_FP64)
    rc, info, lam = c.solve(b, 1e-8, maxit=60)
    check(rc >= 0, f"sphere: solve with the learned stage: {info.iters} iterations")
    c.close()
    # degenerate spheres: one column per panel, one layer
    for kw in (dict(n=1, nlev=2, mg_levels=1), dict(n=2, nlev=1, mg_levels=2)):
        pr = make_sphere(**kw)
        cd = Ctx(lib, pr, omega_rot=pr.omega_rot)
        od = OracleProblem(pr, with_precond=False)
        r_ub, r_pi, b = cd.rhs(4)
        x = np.random.default_rng(2).standard_normal(cd.ntrace)
        y = np.empty(cd.ntrace)
        cd.call("hyb_trace_apply", P(x), P(y))
        ref = od.hyb.S @ x
        rc, info, lam = cd.solve(b, 1e-10)
        check(np.abs(y - ref).max() <= 1e-11 * np.abs(ref).max() and rc == 0 and cd.residual(b, lam) <= 1.01e-10,
              f"sphere C{kw['n']} x {kw['nlev']}: S x against the oracle, FGMRES {info.iters} iterations")
        cd.close()


def mixed_sequence(lib):
    # the unhybridised system (Configuration 1) on a ragged box and a rotating sphere: the mixed
    # right-hand side, operator and approximate-Schur preconditioner against the oracle, FGMRES
    # with restarts, and argument errors
    from oracle.schur import ApproximateSchur, MixedOperator

    for name, prob, kw in (("box", make_box(nx=8, ny=6, nlev=7, dx=5e3, dz=250.0, mg_levels=2, perturb=0.05,
                                            seed=4), {}),
                           ("sphere", make_sphere(4, 5, mg_levels=2, perturb=0.05, seed=3), None)):
        if kw is None:
            kw = dict(omega_rot=prob.omega_rot)
        # restart 30: the first iterations of this method make no progress (a short restart stalls)
        c = Ctx(lib, prob, restart=30, **kw)
        o = OracleProblem(prob)
        op = MixedOperator(o.mixed)
        pc = ApproximateSchur(o.mixed, o.pc.mg.vcycle)
        n = c.ntrace + c.ncell
        r_ub, r_pi, _ = c.rhs(2)
        ruc, rpc = cells_from_soa(r_ub, r_pi)
        b = np.empty(n)
        c.call("hyb_mixed_rhs", P(r_ub), P(r_pi), P(b))
        bref = op.rhs(ruc, rpc)
        check(np.abs(b - bref).max() <= 1e-12 * np.abs(bref).max(), f"{name}: mixed right-hand side against the oracle")
        x = op.expand(np.random.default_rng(5).standard_normal(o.mixed.nu + o.mixed.np_))
        y, z = np.empty(n), np.empty(n)
        c.call("hyb_mixed_apply", P(x), P(y))
        yref = op(x)
        nt = c.ntrace
        eu = np.abs(y[:nt] - yref[:nt]).max() / np.abs(yref[:nt]).max()
        ep = np.abs(y[nt:] - yref[nt:]).max() / np.abs(yref[nt:]).max()
        check(eu <= 1e-11 and ep <= 1e-11, f"{name}: mixed operator against the oracle ({eu:.1e}, {ep:.1e})")
        c.call("hyb_mixed_precondition", P(b), P(z))
        zref = pc(b)
        eu = np.abs(z[:nt] - zref[:nt]).max() / np.abs(zref[:nt]).max()
        ep = np.abs(z[nt:] - zref[nt:]).max() / np.abs(zref[nt:]).max()
        check(eu <= 1e-9 and ep <= 1e-9, f"{name}: approximate-Schur preconditioner against the oracle ({eu:.1e}, {ep:.1e})")
        xs = np.zeros(n)
        hist = (ctypes.c_double * 64)()
        info = N._Info(0, 0, 0, 0.0, ctypes.cast(hist, N._f64p), 64, 0)
        rc = c.call("hyb_mixed_solve", P(b), P(xs), 1e-7, 400, ctypes.byref(info))
        c.call("hyb_mixed_apply", P(xs), P(y))
        res = np.linalg.norm(b - y) / np.linalg.norm(b)
        check(rc == 0 and res <= 1.01e-7,
              f"{name}: mixed FGMRES(30): {info.iters} iterations, {info.restarts} restarts, residual {res:.1e}")
        check(lib.hyb_mixed_solve(c.h, P(b), P(b), 1e-8, 10, None) < 0
              and lib.hyb_mixed_apply(c.h, P(b), P(b)) < 0 and lib.hyb_mixed_precondition(c.h, None, P(z)) < 0,
              f"{name}: aliased or null mixed arguments rejected")
        c.close()


def main():
    lib = N.declare(ctypes.CDLL(sys.argv[1]))
    which = sys.argv[2:] or ["solver", "network", "p1", "sphere", "mixed"]
    if "solver" in which:
        solver_sequence(lib)
    if "network" in which:
        network_sequence(lib)
    if "p1" in which:
        p1_sequence(lib)
    if "sphere" in which:
        sphere_sequence(lib)
    if "mixed" in which:
        mixed_sequence(lib)
    print("sequence complete", flush=True)


if __name__ == "__main__":
    main()
