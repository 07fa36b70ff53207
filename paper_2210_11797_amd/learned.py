"""Learned coarse correction: training data and training loop (driver around the HIP library).

Pairs come from the plain method: from a right-hand side b, the two-level cycle is applied as a
stationary iteration, r_{k+1} = r_k - S M(r_k).  Each step gives one pair from the residual r' left
by the cycle: x = c / s with c = Gamma P^T r' (the coarse right-hand side of Alg. 2) and s = rms(c),
and rhat = P^T r' / s.  Training minimises the error energy that the stage's correction
d = s P (N(x) / H_KK) leaves, through the library's energy loss q^T G q - 2 q^T rhat with
q = N(x) / H_KK and G = P^T S P: no solve with S is needed (see include/hyb.h).

The cycle, S, the restrictions and every network pass (forward, backward, Adam) run in libhyb.so;
torch only holds the vectors and does the vector updates between calls.
"""

from __future__ import annotations

import json

import numpy as np

NTAP = 45
NIN = 3  # input channels: c / s, then the static fields log(h / dz) and z / z_top


def layout(channels=16):
    """(name, shape) of the parameter vector blocks, in order."""
    c = channels
    return [("W1", (c, NIN, NTAP)), ("b1", (c,)), ("W2", (c, c, NTAP)), ("b2", (c,)), ("W3", (1, c, NTAP)),
            ("b3", (1,))]


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
    for co, ci in ((channels, NIN), (channels, channels), (1, channels)):
        W.append(rng.standard_normal((co, ci, NTAP)) * np.sqrt(2.0 / (ci * NTAP)))
        b.append(np.zeros(co))
    W[2] *= 0.1
    return pack(W, b)


def generate_pairs(solver, rhs_list, steps=8):
    """rhs_list: device FP64 trace right-hand sides.  Returns (X FP32, Rhat FP64), both
    [npairs][ncell] on the device."""
    import torch

    n, nc = solver.ntrace, solver.ncell
    X, R = [], []
    z = torch.empty(n, dtype=torch.float64, device="cuda")
    sz = torch.empty_like(z)
    cells = torch.empty(nc, dtype=torch.float64, device="cuda")
    pt = torch.empty_like(cells)
    for b in rhs_list:
        r = b.clone()
        for _ in range(steps):
            solver.precondition(r, z)
            solver.trace_apply(z, sz)
            r -= sz
            solver.restrict(r, cells, 0)
            s = torch.sqrt(torch.mean(cells * cells))
            if not torch.isfinite(s) or float(s) == 0.0:
                break
            solver.restrict(r, pt, 3)
            X.append((cells / s).float())
            R.append(pt / s)
    return torch.stack(X), torch.stack(R)


def train(solver, X, R, steps=1000, batch=8, lr=2e-3, seed=0, log=None):
    """Adam on the energy loss over random mini-batches of pairs; returns the loss history."""
    import torch

    g = torch.Generator(device="cpu").manual_seed(seed)
    npairs = X.shape[0]
    xb = torch.empty((batch, X.shape[1]), dtype=torch.float32, device="cuda")
    rb = torch.empty((batch, R.shape[1]), dtype=torch.float64, device="cuda")
    hist = []
    for it in range(steps):
        idx = torch.randint(0, npairs, (batch,), generator=g).cuda()
        torch.index_select(X, 0, idx, out=xb)
        torch.index_select(R, 0, idx, out=rb)
        loss = solver.nn_energy_train_step(xb, rb, batch, lr)
        hist.append(loss)
        if log and (it % 250 == 0 or it == steps - 1):
            log(f"train step {it}: energy loss {loss:.4e}")
    return hist


def save(path, weights, meta):
    """Weights as a .npz (FP32 vector plus a JSON header string)."""
    np.savez(path, weights=np.asarray(weights, np.float32), meta=np.array(json.dumps(meta)))


def load(path):
    d = np.load(path, allow_pickle=False)
    return d["weights"], json.loads(str(d["meta"]))
