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


def bicgstab(apply_A, apply_M, b, rtol, maxit=200):
    """BiCGStab (van der Vorst, 1992) with right preconditioning M (Saad, Iterative Methods for Sparse
    Linear Systems, Sec. 9.3), from x = 0 until ||b - A x|| <= rtol ||b|| or maxit steps; a breakdown
    (a zero inner product) returns the current iterate.  The coarse solve of the paper's
    Configurations 3a / 3b."""
    x = np.zeros_like(b)
    r = b.copy()
    rh = b.copy()
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    bn = np.linalg.norm(b)
    rho = alpha = omega = 1.0
    rho1 = rh @ r
    for it in range(maxit):
        if bn == 0.0 or rho1 == 0.0 or omega == 0.0:
            break
        beta = (rho1 / rho) * (alpha / omega)
        p = r + (beta if it else 0.0) * (p - omega * v)
        ph = apply_M(p)
        v = apply_A(ph)
        den = rh @ v
        if den == 0.0:
            break
        alpha = rho1 / den
        s = r - alpha * v
        if np.linalg.norm(s) <= rtol * bn:
            x = x + alpha * ph
            break
        sh = apply_M(s)
        t = apply_A(sh)
        tt = t @ t
        omega = (t @ s) / tt if tt > 0.0 else 0.0
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        rho, rho1 = rho1, rh @ r
        if np.linalg.norm(r) <= rtol * bn:
            break
    return x
