"""ctypes binding of libhyb.so (argument marshalling only; every step runs in the HIP library).

The names mirror the C ABI of include/hyb.h.  Device arrays are torch CUDA tensors (FP64,
contiguous); torch provides the memory and the stream, nothing else.  There is no fallback:
if the library is missing or a call fails, an exception is raised.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhyb.so")

HYB_OK = 0
HYB_NOT_CONVERGED = 1
HYB_BREAKDOWN = 2
HYB_DEBUG_ZERO_GAMMA = 1
HYB_DEBUG_NAN_STAGE = 2
HYB_DEBUG_UNPAIRED_RESTRICT = 4
HYB_STAGNATED = 3
PREC_FP64 = 0
PREC_MIXED = 1
PREC_MFMA_FP32 = 2
PREC_MFMA_BF16X = 3
GEOM_BOX = 0
GEOM_SHELL = 1

_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


class _Level(ctypes.Structure):
    _fields_ = [("ncol", ctypes.c_int32), ("col_edge", _i32p), ("edge_col", _i32p), ("edge_lf", _i32p),
                ("parent", _i32p)]


class _Mesh(ctypes.Structure):
    _fields_ = [("nlev", ctypes.c_int32), ("nlevels", ctypes.c_int32), ("levels", ctypes.POINTER(_Level)),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", _f64p), ("order", ctypes.c_int32),
                ("geom", ctypes.c_int32), ("corners", _f64p), ("radius", _f64p)]


class _Params(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("tau_u", ctypes.c_double), ("tau_rho", ctypes.c_double),
                ("tau_theta", ctypes.c_double), ("cp", ctypes.c_double), ("rd", ctypes.c_double),
                ("omega", ctypes.c_double), ("n_pre", ctypes.c_int32), ("n_post", ctypes.c_int32),
                ("omega_p", ctypes.c_double), ("mg_pre", ctypes.c_int32), ("mg_post", ctypes.c_int32),
                ("mg_coarse_sweeps", ctypes.c_int32), ("restart", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("learned", ctypes.c_int32), ("learned_tau", ctypes.c_double),
                ("mg_coarse_cheb", ctypes.c_int32), ("cheb_lo", ctypes.c_double), ("cheb_hi", ctypes.c_double),
                ("omega_rot", ctypes.c_double), ("coarse_mode", ctypes.c_int32), ("coarse_rtol", ctypes.c_double),
                ("smoother_patch", ctypes.c_int32), ("nn_fp32", ctypes.c_int32), ("debug", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("rel_res", ctypes.c_double), ("history", _f64p), ("history_cap", ctypes.c_int32),
                ("history_len", ctypes.c_int32), ("fallbacks", ctypes.c_int32)]


@dataclass
class Params:
    """Solver parameters; defaults are the paper's (Sec. 3.3): omega = 0.6 with 1 pre- and 2
    post-smoothing sweeps, a 4-level pressure multigrid with omega_p = 0.9, 1 pre / 2 post sweeps.
    The paper leaves the coarsest level open: by default 6 steps of the Chebyshev semi-iteration
    over block Jacobi on [cheb_lo, cheb_hi] = [0.02, 2] (mg_coarse_cheb = 0: mg_coarse_sweeps
    damped block-Jacobi sweeps instead)."""

    dt: float = 600.0
    tau_u: float = 0.5
    tau_rho: float = 0.5
    tau_theta: float = 0.5
    cp: float = 1005.0
    rd: float = 287.05
    omega: float = 0.6
    n_pre: int = 1
    n_post: int = 2
    omega_p: float = 0.9
    mg_pre: int = 1
    mg_post: int = 2
    mg_coarse_sweeps: int = 6
    restart: int = 30
    precision: int = PREC_FP64
    learned: int = 0
    learned_tau: float = 3.0
    mg_coarse_cheb: int = 1
    cheb_lo: float = 0.02
    cheb_hi: float = 2.0
    omega_rot: float = 0.0
    coarse_mode: int = 0
    coarse_rtol: float = 1e-2
    smoother_patch: int = 0
    nn_fp32: int = 0
    debug: int = 0

    def to_c(self) -> _Params:
        return _Params(**{f.name: getattr(self, f.name) for f in fields(self)})


ABI_FUNCTIONS = [
    "hyb_create", "hyb_set_params", "hyb_assemble_local", "hyb_condense", "hyb_trace_apply",
    "hyb_precondition", "hyb_solve", "hyb_solve_noalloc", "hyb_recover", "hyb_eliminate", "hyb_back_substitute",
    "hyb_sizes", "hyb_profile", "hyb_profile_family", "hyb_profile_read",
    "hyb_restrict", "hyb_nn_param_count", "hyb_nn_set_weights", "hyb_nn_get_weights", "hyb_nn_forward",
    "hyb_nn_loss_grad", "hyb_nn_train_step", "hyb_nn_energy_grad", "hyb_nn_energy_train_step",
    "hyb_nn_energy_train_step_pairs", "hyb_nn_cycle_pair", "hyb_nn_get_state", "hyb_nn_set_state",
    "hyb_mixed_rhs", "hyb_mixed_apply", "hyb_mixed_precondition", "hyb_mixed_solve",
    "hyb_last_error", "hyb_destroy",
]

_lib = None


def load(path: str = LIB_PATH):
    """Load libhyb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime; it must be loaded first so that this library binds to the
    # same runtime instance (loading libhyb.so first would bring up a second one)
    import torch  # noqa: F401

    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run paper_2210_11797_amd/build.py)")
    _lib = declare(ctypes.CDLL(path))
    return _lib


def declare(lib):
    """Set the ctypes signatures of every entry point of include/hyb.h on a loaded library."""
    vp = ctypes.c_void_p
    lib.hyb_create.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Params), vp, ctypes.POINTER(vp)]
    lib.hyb_set_params.argtypes = [vp, ctypes.POINTER(_Params)]
    lib.hyb_assemble_local.argtypes = [vp, vp, vp, vp, vp]
    lib.hyb_condense.argtypes = [vp, vp, vp, vp]
    lib.hyb_trace_apply.argtypes = [vp, vp, vp]
    lib.hyb_precondition.argtypes = [vp, vp, vp]
    lib.hyb_solve.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(_Info)]
    lib.hyb_solve_noalloc.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(_Info)]
    lib.hyb_recover.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.hyb_eliminate.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.hyb_back_substitute.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.hyb_sizes.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int64)]
    lib.hyb_profile.argtypes = [vp, ctypes.c_int32]
    lib.hyb_profile_family.argtypes = [vp, ctypes.c_char_p]
    lib.hyb_profile_read.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_double)]
    lib.hyb_restrict.argtypes = [vp, vp, vp, ctypes.c_int32]
    lib.hyb_nn_param_count.argtypes = []
    lib.hyb_nn_set_weights.argtypes = [vp, vp, ctypes.c_int64]
    lib.hyb_nn_get_weights.argtypes = [vp, vp, ctypes.c_int64]
    lib.hyb_nn_forward.argtypes = [vp, vp, vp, ctypes.c_int32]
    lib.hyb_nn_loss_grad.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_float), vp]
    lib.hyb_nn_train_step.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_float, ctypes.POINTER(ctypes.c_float)]
    lib.hyb_nn_energy_grad.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), vp]
    lib.hyb_nn_energy_train_step.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_float,
                                             ctypes.POINTER(ctypes.c_double)]
    lib.hyb_nn_energy_train_step_pairs.argtypes = [vp, vp, vp, ctypes.c_int64, vp, ctypes.c_int32, ctypes.c_float,
                                                   ctypes.POINTER(ctypes.c_double)]
    lib.hyb_nn_cycle_pair.argtypes = [vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double)]
    lib.hyb_nn_get_state.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.hyb_nn_set_state.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_int64]
    lib.hyb_mixed_rhs.argtypes = [vp, vp, vp, vp]
    lib.hyb_mixed_apply.argtypes = [vp, vp, vp]
    lib.hyb_mixed_precondition.argtypes = [vp, vp, vp]
    lib.hyb_mixed_solve.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(_Info)]
    lib.hyb_last_error.argtypes = [vp]
    lib.hyb_last_error.restype = ctypes.c_char_p
    lib.hyb_destroy.argtypes = [vp]
    lib.hyb_destroy.restype = None
    for name in ABI_FUNCTIONS:
        if name not in ("hyb_last_error", "hyb_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    return lib


def _ptr(t, n=None, what="array", dtype="float64"):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what}: expected a CUDA tensor")
    if t.dtype != getattr(torch, dtype) or not t.is_contiguous():
        raise TypeError(f"{what}: expected a contiguous {dtype} tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{what}: expected {n} entries, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class HybSolver:
    """One context of the C library for an extruded mesh and its multigrid hierarchy.

    levels: list of dicts (fine to coarse) with ncol, col_edge [4, ncol], edge_col [2, 2ncol],
    edge_lf [2, 2ncol] and, for coarse levels, parent [ncol of the finer level].
    """

    def __init__(self, nlev, levels, dx, dy, dz, params: Params | None = None, stream=None, order: int = 0,
                 corners=None, radius=None):
        import torch

        self.lib = load()
        self.order = int(order)
        # velocity and pressure dofs per cell
        self.nu, self.npr = (6, 1) if self.order == 0 else (36, 8)
        self.params = params or Params()
        self.nlev = int(nlev)
        self._keep = []
        lv = (_Level * len(levels))()
        for i, L in enumerate(levels):
            arrs = {}
            for key in ("col_edge", "edge_col", "edge_lf"):
                a = np.ascontiguousarray(L[key], dtype=np.int32)
                self._keep.append(a)
                arrs[key] = a.ctypes.data_as(_i32p)
            par = None
            if L.get("parent") is not None:
                a = np.ascontiguousarray(L["parent"], dtype=np.int32)
                self._keep.append(a)
                par = a.ctypes.data_as(_i32p)
            lv[i] = _Level(int(L["ncol"]), arrs["col_edge"], arrs["edge_col"], arrs["edge_lf"], par)
        dzh = np.ascontiguousarray(dz, dtype=np.float64)
        self._keep += [lv, dzh]
        geom, cptr, rptr = GEOM_BOX, None, None
        if corners is not None:
            geom = GEOM_SHELL
            ch = np.ascontiguousarray(corners, dtype=np.float64)
            rh = np.ascontiguousarray(radius, dtype=np.float64)
            self._keep += [ch, rh]
            cptr, rptr = ch.ctypes.data_as(_f64p), rh.ctypes.data_as(_f64p)
        mesh = _Mesh(self.nlev, len(levels), lv, float(dx), float(dy), dzh.ctypes.data_as(_f64p), self.order,
                     geom, cptr, rptr)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        cp = self.params.to_c()
        h = ctypes.c_void_p()
        rc = self.lib.hyb_create(ctypes.byref(mesh), ctypes.byref(cp), ctypes.c_void_p(stream.cuda_stream),
                                 ctypes.byref(h))
        if rc != HYB_OK:
            raise RuntimeError(f"hyb_create failed with code {rc}")
        self.h = h
        nt, nc, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self.lib.hyb_sizes(self.h, ctypes.byref(nt), ctypes.byref(nc), ctypes.byref(nb))
        self.ntrace, self.ncell = nt.value, nc.value
        self.ncol = int(levels[0]["ncol"])

    # -- helpers --
    def _check(self, rc, what):
        if rc < 0:
            msg = self.lib.hyb_last_error(self.h).decode()
            raise RuntimeError(f"{what} failed ({rc}): {msg}")
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.hyb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self):
        nb = ctypes.c_int64()
        self.lib.hyb_sizes(self.h, None, None, ctypes.byref(nb))
        return nb.value

    # -- ABI calls --
    def set_params(self, params: Params):
        cp = params.to_c()
        self._check(self.lib.hyb_set_params(self.h, ctypes.byref(cp)), "hyb_set_params")
        self.params = params

    def assemble_local(self, theta_w, exner_hat_w, exner_c, rho_c):
        nw, nc = (self.nlev + 1) * self.ncol, self.ncell
        self._check(self.lib.hyb_assemble_local(self.h, _ptr(theta_w, nw, "theta_w"),
                                                _ptr(exner_hat_w, nw, "exner_hat_w"),
                                                _ptr(exner_c, nc, "exner_c"), _ptr(rho_c, nc, "rho_c")),
                    "hyb_assemble_local")

    def condense(self, r_ub=None, r_pi=None, b_lambda=None):
        if r_ub is None:
            self._check(self.lib.hyb_condense(self.h, None, None, None), "hyb_condense")
            return
        self._check(self.lib.hyb_condense(self.h, _ptr(r_ub, self.nu * self.ncell, "r_ub"),
                                          _ptr(r_pi, self.npr * self.ncell, "r_pi"),
                                          _ptr(b_lambda, self.ntrace, "b_lambda")), "hyb_condense")

    def trace_apply(self, x, y):
        self._check(self.lib.hyb_trace_apply(self.h, _ptr(x, self.ntrace, "x"), _ptr(y, self.ntrace, "y")),
                    "hyb_trace_apply")

    def precondition(self, r, z):
        self._check(self.lib.hyb_precondition(self.h, _ptr(r, self.ntrace, "r"), _ptr(z, self.ntrace, "z")),
                    "hyb_precondition")

    # the unhybridised system (the paper's Configuration 1): vectors of ntrace + ncell doubles
    @property
    def nmixed(self):
        return self.ntrace + self.ncell

    def mixed_rhs(self, r_ub, r_pi, b):
        self._check(self.lib.hyb_mixed_rhs(self.h, _ptr(r_ub, 6 * self.ncell, "r_ub"), _ptr(r_pi, self.ncell, "r_pi"),
                                           _ptr(b, self.nmixed, "b")), "hyb_mixed_rhs")

    def mixed_apply(self, x, y):
        self._check(self.lib.hyb_mixed_apply(self.h, _ptr(x, self.nmixed, "x"), _ptr(y, self.nmixed, "y")),
                    "hyb_mixed_apply")

    def mixed_precondition(self, r, z):
        self._check(self.lib.hyb_mixed_precondition(self.h, _ptr(r, self.nmixed, "r"), _ptr(z, self.nmixed, "z")),
                    "hyb_mixed_precondition")

    def mixed_solve(self, b, x, rtol=1e-8, maxit=500, history=256):
        hist = (ctypes.c_double * max(1, history))()
        info = _Info(0, 0, 0, 0.0, ctypes.cast(hist, _f64p), history, 0)
        rc = self._check(self.lib.hyb_mixed_solve(self.h, _ptr(b, self.nmixed, "b"), _ptr(x, self.nmixed, "x"),
                                                  float(rtol), int(maxit), ctypes.byref(info)), "hyb_mixed_solve")
        return dict(status=rc, iters=info.iters, restarts=info.restarts, rel_res=info.rel_res,
                    history=[hist[i] for i in range(info.history_len)])

    def solve(self, b_lambda, lam, rtol=1e-8, maxit=500, history=256, noalloc=False):
        """hyb_solve, or with noalloc=True hyb_solve_noalloc (no allocation during the call)."""
        hist = (ctypes.c_double * max(1, history))()
        info = _Info(0, 0, 0, 0.0, ctypes.cast(hist, _f64p), history, 0)
        name = "hyb_solve_noalloc" if noalloc else "hyb_solve"
        rc = self._check(getattr(self.lib, name)(self.h, _ptr(b_lambda, self.ntrace, "b_lambda"),
                                                 _ptr(lam, self.ntrace, "lambda"), float(rtol), int(maxit),
                                                 ctypes.byref(info)), name)
        return dict(status=rc, iters=info.iters, restarts=info.restarts, rel_res=info.rel_res,
                    history=[hist[i] for i in range(info.history_len)], fallbacks=info.fallbacks)

    def recover(self, r_ub, r_pi, lam, u_b, pi):
        self._check(self.lib.hyb_recover(self.h, _ptr(r_ub, self.nu * self.ncell, "r_ub"),
                                         _ptr(r_pi, self.npr * self.ncell, "r_pi"), _ptr(lam, self.ntrace, "lambda"),
                                         _ptr(u_b, self.nu * self.ncell, "u_b"), _ptr(pi, self.npr * self.ncell, "pi")),
                    "hyb_recover")

    def eliminate(self, r_ub, r_rho, r_theta, r_pi, r_ub_bar, r_pi_bar):
        """hyb_eliminate: the 2x2 right-hand sides from the four residuals (theta' and rho' eliminated)."""
        nc, ncol = self.ncell, self.ncol
        self._check(self.lib.hyb_eliminate(self.h, _ptr(r_ub, 6 * nc, "r_ub"), _ptr(r_rho, nc, "r_rho"),
                                           _ptr(r_theta, nc + ncol, "r_theta"), _ptr(r_pi, nc, "r_pi"),
                                           _ptr(r_ub_bar, 6 * nc, "r_ub_bar"), _ptr(r_pi_bar, nc, "r_pi_bar")),
                    "hyb_eliminate")

    def back_substitute(self, r_rho, r_theta, u_b, rho, theta):
        """hyb_back_substitute: rho' and theta' (each cell's bottom and top node) from the velocity."""
        nc, ncol = self.ncell, self.ncol
        self._check(self.lib.hyb_back_substitute(self.h, _ptr(r_rho, nc, "r_rho"), _ptr(r_theta, nc + ncol, "r_theta"),
                                                 _ptr(u_b, 6 * nc, "u_b"), _ptr(rho, nc, "rho"),
                                                 _ptr(theta, 2 * nc, "theta")),
                    "hyb_back_substitute")

    def restrict(self, r, cells, mode=0):
        self._check(self.lib.hyb_restrict(self.h, _ptr(r, self.ntrace, "r"), _ptr(cells, self.ncell, "cells"),
                                          int(mode)), "hyb_restrict")

    # -- learned coarse correction --
    def nn_param_count(self):
        return int(self.lib.hyb_nn_param_count())

    def nn_set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._check(self.lib.hyb_nn_set_weights(self.h, w.ctypes.data_as(ctypes.c_void_p), w.size),
                    "hyb_nn_set_weights")

    def nn_get_weights(self):
        w = np.empty(self.nn_param_count(), np.float32)
        self._check(self.lib.hyb_nn_get_weights(self.h, w.ctypes.data_as(ctypes.c_void_p), w.size),
                    "hyb_nn_get_weights")
        return w

    def nn_forward(self, x, y, nsamp=1):
        n = self.ncell * nsamp
        self._check(self.lib.hyb_nn_forward(self.h, _ptr(x, n, "x", "float32"), _ptr(y, n, "y", "float32"),
                                            int(nsamp)), "hyb_nn_forward")

    def nn_loss_grad(self, x, t, nsamp=1, want_grad=True):
        n = self.ncell * nsamp
        loss = ctypes.c_float()
        g = np.empty(self.nn_param_count(), np.float32) if want_grad else None
        self._check(self.lib.hyb_nn_loss_grad(self.h, _ptr(x, n, "x", "float32"), _ptr(t, n, "t", "float32"),
                                              int(nsamp), ctypes.byref(loss),
                                              g.ctypes.data_as(ctypes.c_void_p) if g is not None else None),
                    "hyb_nn_loss_grad")
        return loss.value, g

    def nn_train_step(self, x, t, nsamp, lr):
        n = self.ncell * nsamp
        loss = ctypes.c_float()
        self._check(self.lib.hyb_nn_train_step(self.h, _ptr(x, n, "x", "float32"), _ptr(t, n, "t", "float32"),
                                               int(nsamp), float(lr), ctypes.byref(loss)), "hyb_nn_train_step")
        return loss.value

    def nn_energy_grad(self, x, rhat, nsamp=1, want_grad=True):
        n = self.ncell * nsamp
        loss = ctypes.c_double()
        g = np.empty(self.nn_param_count(), np.float32) if want_grad else None
        self._check(self.lib.hyb_nn_energy_grad(self.h, _ptr(x, n, "x", "float32"), _ptr(rhat, n, "rhat"),
                                                int(nsamp), ctypes.byref(loss),
                                                g.ctypes.data_as(ctypes.c_void_p) if g is not None else None),
                    "hyb_nn_energy_grad")
        return loss.value, g

    def nn_energy_train_step(self, x, rhat, nsamp, lr):
        n = self.ncell * nsamp
        loss = ctypes.c_double()
        self._check(self.lib.hyb_nn_energy_train_step(self.h, _ptr(x, n, "x", "float32"), _ptr(rhat, n, "rhat"),
                                                      int(nsamp), float(lr), ctypes.byref(loss)),
                    "hyb_nn_energy_train_step")
        return loss.value

    def nn_energy_train_step_pairs(self, X, R, idx, lr):
        """One Adam step on the pairs idx (host ints) of X [npairs, ncell] (FP32) and R (FP64)."""
        npairs = X.shape[0]
        n = self.ncell * npairs
        sel = np.ascontiguousarray(idx, dtype=np.int32)
        loss = ctypes.c_double()
        self._check(self.lib.hyb_nn_energy_train_step_pairs(
            self.h, _ptr(X, n, "X", "float32"), _ptr(R, n, "R"), int(npairs), sel.ctypes.data_as(ctypes.c_void_p),
            int(sel.size), float(lr), ctypes.byref(loss)), "hyb_nn_energy_train_step_pairs")
        return loss.value

    def nn_get_state(self):
        """(m, v, step): the Adam moments (FP32) and step count of the training."""
        n = self.nn_param_count()
        m, v, step = np.empty(n, np.float32), np.empty(n, np.float32), ctypes.c_int64()
        self._check(self.lib.hyb_nn_get_state(self.h, m.ctypes.data_as(ctypes.c_void_p),
                                              v.ctypes.data_as(ctypes.c_void_p), n, ctypes.byref(step)),
                    "hyb_nn_get_state")
        return m, v, step.value

    def nn_set_state(self, m, v, step):
        m = np.ascontiguousarray(m, dtype=np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        self._check(self.lib.hyb_nn_set_state(self.h, m.ctypes.data_as(ctypes.c_void_p),
                                              v.ctypes.data_as(ctypes.c_void_p), m.size, int(step)),
                    "hyb_nn_set_state")

    def nn_cycle_pair(self, r, x, rhat):
        """One cycle step on r (in place) and its training pair into x (FP32) and rhat; returns the
        scale s, or None when the residual's coarse part vanished (HYB_BREAKDOWN)."""
        s = ctypes.c_double()
        rc = self.lib.hyb_nn_cycle_pair(self.h, _ptr(r, self.ntrace, "r"), _ptr(x, self.ncell, "x", "float32"),
                                        _ptr(rhat, self.ncell, "rhat"), ctypes.byref(s))
        if rc == HYB_BREAKDOWN:
            return None
        self._check(rc, "hyb_nn_cycle_pair")
        return s.value

    def profile(self, enable: bool):
        self._check(self.lib.hyb_profile(self.h, 1 if enable else 0), "hyb_profile")

    def profile_family(self, family: str):
        """Record HIP events around the launches of one kernel family only."""
        self._check(self.lib.hyb_profile_family(self.h, family.encode()), "hyb_profile_family")

    def profile_read(self, family: str):
        n, ms = ctypes.c_int64(), ctypes.c_double()
        self._check(self.lib.hyb_profile_read(self.h, family.encode(), ctypes.byref(n), ctypes.byref(ms)),
                    "hyb_profile_read")
        return n.value, ms.value


def solver_for(prob, params: Params | None = None, order: int = 0, stream=None) -> "HybSolver":
    """A HybSolver for a synthetic problem: the periodic box, or the extruded cubed sphere (its
    corner unit vectors and interface radii as the shell geometry)."""
    if getattr(prob, "geom", "box") == "shell":
        return HybSolver(prob.nlev, levels_of(prob), 0.0, 0.0, prob.dz, params, stream=stream, order=order,
                         corners=prob.corners, radius=prob.radius)
    return HybSolver(prob.nlev, levels_of(prob), prob.dx, prob.dy, prob.dz, params, stream=stream, order=order)


def levels_of(prob):
    """Mesh hierarchy of a synthetic problem as the dicts HybSolver takes."""
    out = []
    for i, L in enumerate(prob.levels):
        out.append(dict(ncol=L.ncol, col_edge=L.col_edge, edge_col=L.edge_col, edge_lf=L.edge_lf,
                        parent=None if i == 0 else L.parent))
    return out
