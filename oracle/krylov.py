"""Flexible GMRES (test infrastructure).

Right-preconditioned flexible GMRES (Saad, 1993): the preconditioned vectors
z_j = M(v_j) are kept, Arnoldi uses modified Gram-Schmidt, and the
least-squares problem min || beta e_1 - Hbar y || is solved with
``numpy.linalg.lstsq`` at every step, whose residual norm is the stopping
test ||b - A x|| / ||b|| (the paper's relative residual, Sec. 3.4).  Restart
after ``restart`` steps from the current iterate.

Parity: with a fixed linear preconditioner the iterates equal those of
right-preconditioned GMRES; pinned in the tests by the minimal-residual
property over an explicitly built Krylov basis.
"""

from __future__ import annotations

import numpy as np


def fgmres(apply_A, apply_M, b, x0=None, rtol=1e-8, restart=30, maxit=500):
    """Returns (x, history of relative residuals, iterations, converged)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), [0.0], 0, True
    hist = []
    its = 0
    r = b - apply_A(x)
    beta = np.linalg.norm(r)
    hist.append(beta / bnorm)
    while its < maxit:
        if beta / bnorm <= rtol:
            return x, hist, its, True
        V = [r / beta]
        Z = []
        Hb = np.zeros((restart + 1, restart))
        y = np.zeros(0)
        for j in range(restart):
            z = apply_M(V[j])
            w = apply_A(z)
            Z.append(z)
            for i in range(j + 1):
                Hb[i, j] = np.dot(w, V[i])
                w = w - Hb[i, j] * V[i]
            Hb[j + 1, j] = np.linalg.norm(w)
            e1 = np.zeros(j + 2)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(Hb[: j + 2, : j + 1], e1, rcond=None)
            res = np.linalg.norm(e1 - Hb[: j + 2, : j + 1] @ y)
            its += 1
            hist.append(res / bnorm)
            if res / bnorm <= rtol or its >= maxit or Hb[j + 1, j] == 0.0:
                break
            V.append(w / Hb[j + 1, j])
        x = x + np.array(Z).T @ y
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= rtol:
            return x, hist, its, True
    return x, hist, its, beta / bnorm <= rtol
