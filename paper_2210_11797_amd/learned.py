"""Learned coarse correction: training data and training loop (driver around the HIP library).

Pairs (input, target) come from the plain method: for a right-hand side b, lambda* is solved to a
tight tolerance; then the two-level cycle is applied as a stationary iteration, x_{k+1} = x_k +
M(r_k), r_{k+1} = r_k - S M(r_k).  Each step gives one pair with the residual r' = r_{k+1} left by
the cycle: input c / s with c = Gamma P^T r' (the coarse right-hand side of Alg. 2) and s = rms(c);
target the facet average of the remaining error lambda* - x_{k+1}, divided by s.  At inference the
library adds s P N(c / s) to the output of the cycle (see include/hyb.h).

The solves, the cycle, S, the restrictions and every network pass (forward, backward, Adam) run in
libhyb.so; torch only holds the vectors and does the vector updates between calls.
"""

from __future__ import annotations

import json

import numpy as np

NTAP = 45


def layout(channels=16):
    """(name, shape) of the parameter vector blocks, in order."""
    c = channels
    return [("W1", (c, 1, NTAP)), ("b1", (c,)), ("W2", (c, c, NTAP)), ("b2", (c,)), ("W3", (1, c, NTAP)), ("b3", (1,))]


def pack(W, b):
    return np.concatenate([W[0].ravel(), b[0], W[1].ravel(), b[1], W[2].ravel(), b[2]]).astype(np.float32)


def unpack(vec, channels=16):
    out, off = {}, 0
    for name, shp in layout(channels):
        n = int(np.prod(shp))
        out[name] = np.asarray(vec[off : off + n], dtype=np.float64).reshape(shp)
        off += n
    return [out["W1"], out["W2"], out["W3"]], [out["b1"], out["b2"], out["b3"]]


def init_params(channels=16, seed=0):
    """He-scaled random weights, zero biases, a small last layer (FP32 vector)."""
    rng = np.random.default_rng(seed)
    W, b = [], []
    for co, ci in ((channels, 1), (channels, channels), (1, channels)):
        W.append(rng.standard_normal((co, ci, NTAP)) * np.sqrt(2.0 / (ci * NTAP)))
        b.append(np.zeros(co))
    W[2] *= 0.1
    return pack(W, b)


def generate_pairs(solver, rhs_list, steps=8, rtol=1e-12):
    """rhs_list: device FP64 trace right-hand sides.  Returns (X, T) device FP32 [npairs][ncell]."""
    import torch

    n, nc = solver.ntrace, solver.ncell
    X, T = [], []
    lam_star = torch.zeros(n, dtype=torch.float64, device="cuda")
    z = torch.empty_like(lam_star)
    sz = torch.empty_like(lam_star)
    cells = torch.empty(nc, dtype=torch.float64, device="cuda")
    err_cells = torch.empty_like(cells)
    for b in rhs_list:
        lam_star.zero_()
        info = solver.solve(b, lam_star, rtol=rtol, maxit=400)
        if info["status"] != 0:
            raise RuntimeError(f"training solve did not converge: {info}")
        x = torch.zeros_like(lam_star)
        r = b.clone()
        for _ in range(steps):
            solver.precondition(r, z)
            x += z
            solver.trace_apply(z, sz)
            r -= sz
            solver.restrict(r, cells, 0)
            s = torch.sqrt(torch.mean(cells * cells))
            if not torch.isfinite(s) or float(s) == 0.0:
                break
            solver.restrict(lam_star - x, err_cells, 1)
            X.append((cells / s).float())
            T.append((err_cells / s).float())
    return torch.stack(X), torch.stack(T)


def train(solver, X, T, steps=300, batch=8, lr=1e-3, seed=0, log=None):
    """Adam on random mini-batches of pairs; returns the loss history."""
    import torch

    g = torch.Generator(device="cpu").manual_seed(seed)
    npairs = X.shape[0]
    xb = torch.empty((batch, X.shape[1]), dtype=torch.float32, device="cuda")
    tb = torch.empty_like(xb)
    hist = []
    for it in range(steps):
        idx = torch.randint(0, npairs, (batch,), generator=g).cuda()
        torch.index_select(X, 0, idx, out=xb)
        torch.index_select(T, 0, idx, out=tb)
        loss = solver.nn_train_step(xb, tb, batch, lr)
        hist.append(loss)
        if log and (it % 50 == 0 or it == steps - 1):
            log(f"train step {it}: loss {loss:.4e}")
    return hist


def save(path, weights, meta):
    """Weights as a .npz (FP32 vector plus a JSON header string)."""
    np.savez(path, weights=np.asarray(weights, np.float32), meta=np.array(json.dumps(meta)))


def load(path):
    d = np.load(path, allow_pickle=False)
    return d["weights"], json.loads(str(d["meta"]))
