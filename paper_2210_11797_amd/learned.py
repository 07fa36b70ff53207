"""Learned coarse correction: training data and training loop (driver around the HIP library).

Pairs come from the plain method: from a right-hand side b, the two-level cycle is applied as a
stationary iteration, r_{k+1} = r_k - S M(r_k).  Each step gives one pair from the residual r' left
by the cycle: x = c / s with c = Gamma P^T r' (the coarse right-hand side of Alg. 2) and s = rms(c),
and rhat = P^T r' / s.  Training minimises the error energy that the stage's correction
d = s P (N(x) / H_KK) leaves, through the library's energy loss q^T G q - 2 q^T rhat with
q = N(x) / H_KK and G = P^T S P: no solve with S is needed (see include/hyb.h).

The cycle, S, the restrictions, the residual update and normalisation of a pair
(hyb_nn_cycle_pair), the gathering of a mini-batch and every network pass (forward, backward, Adam)
run in libhyb.so; torch only holds the vectors.
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
    [npairs][ncell] on the device; each right-hand side gives up to ``steps`` pairs
    (hyb_nn_cycle_pair: the cycle step, the residual update and the normalisation run in the
    library)."""
    import torch

    X, R = [], []
    for b in rhs_list:
        r = b.clone()
        for _ in range(steps):
            x = torch.empty(solver.ncell, dtype=torch.float32, device="cuda")
            rh = torch.empty(solver.ncell, dtype=torch.float64, device="cuda")
            if solver.nn_cycle_pair(r, x, rh) is None:
                break
            X.append(x)
            R.append(rh)
    return torch.stack(X), torch.stack(R)


def train(solver, X, R, steps=1000, batch=8, lr=2e-3, seed=0, log=None):
    """Adam on the energy loss over random mini-batches of pairs (gathered inside the library);
    returns the loss history."""
    rng = np.random.default_rng(seed)
    npairs = X.shape[0]
    hist = []
    for it in range(steps):
        loss = solver.nn_energy_train_step_pairs(X, R, rng.integers(0, npairs, batch), lr)
        hist.append(loss)
        if log and (it % 250 == 0 or it == steps - 1):
            log(f"train step {it}: energy loss {loss:.4e}")
    return hist


def train_streaming(solver, next_rhs, npairs=4096, pool=256, steps_per_rhs=8, batch=8, lr=2e-3, updates=1000,
                    seed=0, log=None):
    """Training on pairs generated on the fly, for meshes where all pairs do not fit in memory:
    a pool of ``pool`` pairs is refilled from new right-hand sides (``next_rhs()``, each giving
    ``steps_per_rhs`` pairs of the cycle iteration) until ``npairs`` pairs have been made, and
    ``updates`` Adam steps on random mini-batches of the pool are spread over the refills.
    Returns (loss history, pairs made)."""
    import torch

    rng = np.random.default_rng(seed)
    nc = solver.ncell
    X = torch.empty((pool, nc), dtype=torch.float32, device="cuda")
    R = torch.empty((pool, nc), dtype=torch.float64, device="cuda")
    made, filled, slot, done, hist = 0, 0, 0, 0, []
    while made < npairs:
        r = next_rhs().clone()
        for _ in range(steps_per_rhs):
            if made >= npairs or solver.nn_cycle_pair(r, X[slot], R[slot]) is None:
                break
            made += 1
            filled = min(pool, filled + 1)
            slot = (slot + 1) % pool
        if filled < min(pool, npairs):
            continue
        target = updates * made // npairs
        while done < target:
            hist.append(solver.nn_energy_train_step_pairs(X[:filled], R[:filled], rng.integers(0, filled, batch), lr))
            if log and (done % 50 == 0 or done == updates - 1):
                log(f"train step {done} ({made} pairs made): energy loss {hist[-1]:.4e}")
            done += 1
    return hist, made


def save(path, weights, meta, state=None):
    """Weights as a .npz (FP32 vector plus a JSON header string: shape, seed, loss, ...); with
    state = (m, v, step) from HybSolver.nn_get_state also the Adam moments, so that training can
    resume (``resume``)."""
    arrays = dict(weights=np.asarray(weights, np.float32), meta=np.array(json.dumps(meta)))
    if state is not None:
        m, v, step = state
        arrays.update(adam_m=np.asarray(m, np.float32), adam_v=np.asarray(v, np.float32),
                      adam_step=np.array(int(step), np.int64))
    np.savez(path, **arrays)


def load(path):
    """(weights, meta, state): state = (m, v, step), or None when the file has no Adam state."""
    d = np.load(path, allow_pickle=False)
    state = None
    if "adam_m" in d.files:
        state = (d["adam_m"], d["adam_v"], int(d["adam_step"]))
    return d["weights"], json.loads(str(d["meta"])), state


def resume(solver, path):
    """Load weights and, if saved, the Adam state into a context, to continue training there."""
    w, meta, state = load(path)
    solver.nn_set_weights(w)
    if state is not None:
        solver.nn_set_state(*state)
    return meta
