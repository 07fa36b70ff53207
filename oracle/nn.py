"""Learned coarse correction network and stage (test infrastructure, FP64 NumPy reference).

The network maps a DG0 field (one value per cell, [L][ncol]), with two static fields of the mesh
beside it (log(h / dz), h = sqrt(|K| / dz) the cell's horizontal size, and the cell-centre height
over the lid's), to a DG0 field through three 3D convolutions, 3 -> C -> C -> 1 channels, each tap set being the 3 x 3 horizontal neighbourhood of a
column (the column, its four edge neighbours and four corner neighbours) times 5 vertical offsets
(-2..2, zero padded above the lid and below the ground); ReLU after the first two layers.  On the
cubed sphere the neighbourhood follows each column's frame across panel edges, and the corner
neighbour that does not exist at a cube vertex is zero padded.

The stage (not part of the paper) follows the two-level cycle z = M(v) of Alg. 2: with the residual
r' = v - S z it left, the coarse right-hand side c = Gamma P^T r' of Alg. 2 and s = rms(c), the
network proposes d = s P (N(c / s) / H_KK) (H_KK the diagonal of the pressure operator, which makes
the network's target dimensionless), and the FP64 residual decides: z + d is kept only if
||r' - S d|| < tau ||r'||, else z (also when N's output is not finite).

Training minimises the error energy left after the correction.  With e' = S^-1 r' and the
correction P delta, delta = s q, q = N(x) / H_KK, the energy changes by
    (e' - P delta)^T S (e' - P delta) - e'^T S e' = delta^T G delta - 2 delta^T P^T r'   (S symmetric)
with G = P^T S P, so the loss per pair is q^T G q - 2 q^T rhat, rhat = P^T r' / s: it needs r' and
applications of G only, never S^-1.  Pairs (x = c / s, rhat) come from the plain method's
stationary iteration.

Parity: the network is pinned by central finite differences of the loss with respect to every
weight group and the input, by translation equivariance on the periodic box, and by one-hot weights
that must reproduce shifted copies of the input; the stage by an exact identity network (the
correction must equal the closed form P H_KK^-1 Gamma P^T r'), by positive homogeneity of degree one
in (v, z), and by networks that must be rejected (zero output; a correction far too large); the
energy loss by central finite differences and, in the symmetric case, by the error energies
computed with a direct solve.
"""

from __future__ import annotations

import numpy as np

NH = 9  # horizontal taps: centre, W, E, S, N, SW, SE, NW, NE
NV = 5  # vertical taps: dk = -2..2
NT = NH * NV
# horizontal direction of each tap and its opposite
H_OFFSETS = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1), (-1, -1), (1, -1), (-1, 1), (1, 1)]


def neighbour_table(nx, ny):
    """nb[h][col] = column at horizontal offset H_OFFSETS[h] on the periodic nx x ny box."""
    col = np.arange(nx * ny)
    ix, iy = col % nx, col // nx
    return np.stack([((iy + dy) % ny) * nx + (ix + dx) % nx for (dx, dy) in H_OFFSETS]).astype(np.int64)


# directions counter-clockwise in a column's frame (E, N, W, S) and the local faces W, E, S, N
_DIR_OF_FACE = np.array([2, 0, 3, 1])
_FACE_OF_DIR = np.array([1, 3, 0, 2])


def neighbour_table_from_tables(col_edge, edge_col, edge_lf):
    """nb[h][col] for any quadrilateral mesh whose column frames turn the same way (the cubed
    sphere): the edge neighbours across W, E, S, N, and the corner neighbour at offset (dx, dy)
    reached by one step along y and then one along x, the x direction carried into the
    neighbour's frame by the quarter turn that maps the step's direction onto the neighbour's
    face pointing away from the column.  Where the two orders of the steps disagree (the three
    columns at a cube vertex have no corner neighbour there) the entry is -1 (zero padded)."""
    ce, ec, el = (np.asarray(a, np.int64) for a in (col_edge, edge_col, edge_lf))
    ncol = ce.shape[1]
    col = np.arange(ncol)
    nbr = np.empty((4, ncol), np.int64)
    nlf = np.empty((4, ncol), np.int64)
    for f in range(4):
        e = ce[f]
        side = np.where((ec[0, e] == col) & (el[0, e] == f), 0, 1)
        nbr[f] = ec[1 - side, e]
        nlf[f] = el[1 - side, e]

    def route(f1, f2):
        n = nbr[f1]
        turn = (_DIR_OF_FACE[nlf[f1]] + 2 - _DIR_OF_FACE[f1]) % 4
        return nbr[_FACE_OF_DIR[(_DIR_OF_FACE[f2] + turn) % 4], n]

    def corner(fx, fy):
        a, b = route(fy, fx), route(fx, fy)
        return np.where(a == b, a, -1)

    W, E, S, N = 0, 1, 2, 3
    return np.stack([col, nbr[W], nbr[E], nbr[S], nbr[N], corner(W, S), corner(E, S), corner(W, N),
                     corner(E, N)]).astype(np.int64)


NIN = 3  # input channels: the normalised coarse residual, log(h / dz), z / z_top


def static_inputs(vol, z, ncol):
    """The two static input channels (2, L*ncol) of the network: log(h / dz) with h = sqrt(|K| / dz)
    the cell's horizontal size, and the height of the cell centre over that of the lid.
    vol: cell volumes (L*ncol,); z: interface heights (L+1,)."""
    z = np.asarray(z, np.float64)
    nlev = z.shape[0] - 1
    k = np.arange(nlev * ncol) // ncol
    dz = (z[1:] - z[:-1])[k]
    h = np.sqrt(np.asarray(vol, np.float64) / dz)
    zc = (0.5 * (z[1:] + z[:-1]) - z[0])[k] / (z[-1] - z[0])
    return np.stack([np.log(h / dz), zc])


def init_weights(channels=16, seed=0):
    rng = np.random.default_rng(seed)
    shapes = [(channels, NIN), (channels, channels), (1, channels)]
    W, b = [], []
    for co, ci in shapes:
        fan_in = ci * NT
        W.append(rng.standard_normal((co, ci, NT)) * np.sqrt(2.0 / fan_in))
        b.append(np.zeros(co))
    W[-1] *= 0.1
    return W, b


def conv(x, W, bias, nb, nlev):
    """x: (ci, L*ncol) -> (co, L*ncol); y[co, k, c] = b[co] + sum W[co, ci, t] x[ci, k+dk, nb[h, c]]."""
    ci, n = x.shape
    ncol = n // nlev
    co = W.shape[0]
    xr = x.reshape(ci, nlev, ncol)
    y = np.repeat(bias[:, None], n, axis=1).reshape(co, nlev, ncol).copy()
    for h in range(NH):
        ok = nb[h] >= 0  # a missing neighbour (cube vertex) reads zeros
        xh = xr[:, :, np.where(ok, nb[h], 0)] * ok  # (ci, L, ncol): value at the neighbour column
        for v in range(NV):
            dk = v - 2
            shifted = np.zeros_like(xh)
            if dk >= 0:
                shifted[:, : nlev - dk] = xh[:, dk:]
            else:
                shifted[:, -dk:] = xh[:, : nlev + dk]
            y += np.einsum("oi,ilc->olc", W[:, :, h * NV + v], shifted)
    return y.reshape(co, n)


def conv_grads(x, W, dy, nb, nlev):
    """Gradients of sum(dy * conv(x)) with respect to x, W and the bias."""
    ci, n = x.shape
    ncol = n // nlev
    co = W.shape[0]
    xr = x.reshape(ci, nlev, ncol)
    dyr = dy.reshape(co, nlev, ncol)
    dW = np.zeros_like(W)
    dx = np.zeros((ci, nlev, ncol))
    for h in range(NH):
        ok = nb[h] >= 0
        xh = xr[:, :, np.where(ok, nb[h], 0)] * ok
        for v in range(NV):
            dk = v - 2
            shifted = np.zeros_like(xh)
            if dk >= 0:
                shifted[:, : nlev - dk] = xh[:, dk:]
            else:
                shifted[:, -dk:] = xh[:, : nlev + dk]
            dW[:, :, h * NV + v] = np.einsum("olc,ilc->oi", dyr, shifted)
            # transpose: contribution W^T dy placed back at (k + dk, nb[h, c])
            g = np.einsum("oi,olc->ilc", W[:, :, h * NV + v], dyr)
            back = np.zeros_like(g)
            if dk >= 0:
                back[:, dk:] = g[:, : nlev - dk]
            else:
                back[:, : nlev + dk] = g[:, -dk:]
            np.add.at(dx, (slice(None), slice(None), nb[h][ok]), back[:, :, ok])
    return dx.reshape(ci, n), dW, dyr.sum(axis=(1, 2))


def forward(x, W, b, nb, nlev, static=None):
    """Returns the output and the post-activation values of every layer (x is (L*ncol,)), in FP64;
    static: the static input channels (zeros if None)."""
    nst = W[0].shape[1] - 1
    if nst == 0:
        acts = [x[None, :]]
    else:
        if static is None:
            static = np.zeros((nst, x.shape[0]))
        acts = [np.vstack([x[None, :], np.asarray(static, np.float64).reshape(nst, -1)])]
    h = acts[0]
    for i in range(3):
        h = conv(h, W[i], b[i], nb, nlev)
        if i < 2:
            h = np.maximum(h, 0.0)
        acts.append(h)
    return h[0], acts


def loss_and_grads(x, target, W, b, nb, nlev, static=None):
    """Mean squared error over cells and its gradients (dW list, db list, dx)."""
    y, acts = forward(x, W, b, nb, nlev, static=static)
    n = y.shape[0]
    diff = y - target
    loss = float(np.mean(diff * diff))
    dy = (2.0 / n) * diff[None, :]
    dWs, dbs = [None] * 3, [None] * 3
    for i in (2, 1, 0):
        if i < 2:
            dy = dy * (acts[i + 1] > 0.0)
        dx, dWs[i], dbs[i] = conv_grads(acts[i], W[i], dy, nb, nlev)
        dy = dx
    return loss, dWs, dbs, dy[0]


def bf16_round(a):
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def learned_correction(v, z, S, P, gamma, hdiag, W, b, nb, nlev, tau=3.0, static=None):
    """The learned stage after z = M(v).  Returns (z_new, accepted)."""
    rp = v - S @ z
    c = gamma * (P.T @ rp)
    s = float(np.sqrt(np.mean(c * c)))
    x = c / s if s > 0.0 else np.zeros_like(c)
    y, _ = forward(x, W, b, nb, nlev, static=static)
    if not np.all(np.isfinite(y)):
        return z, False
    d = s * (P @ (y / hdiag))
    if np.linalg.norm(rp - S @ d) < tau * np.linalg.norm(rp):
        return z + d, True
    return z, False


def identity_weights(channels=16):
    """Weights for which the network is exactly the identity: channel 0 carries relu(x), channel 1
    relu(-x), the last layer returns their difference (centre tap, dk = 0, zero biases)."""
    W = [np.zeros((channels, NIN, NT)), np.zeros((channels, channels, NT)), np.zeros((1, channels, NT))]
    centre = 0 * NV + 2
    W[0][0, 0, centre], W[0][1, 0, centre] = 1.0, -1.0
    W[1][0, 0, centre], W[1][1, 1, centre] = 1.0, 1.0
    W[2][0, 0, centre], W[2][0, 1, centre] = 1.0, -1.0
    return W, [np.zeros(channels), np.zeros(channels), np.zeros(1)]


def energy_loss_and_grads(x, rhat, W, b, nb, nlev, G, hdiag, static=None):
    """Energy loss of one pair and its gradients (dW list, db list).

    q = N(x) / H_KK,  loss = (q^T G q - 2 q^T rhat) * mean(H_KK) / ncell  (the scale makes the loss
    dimensionless and of order one; averaging over a batch is the caller's)."""
    y, acts = forward(x, W, b, nb, nlev, static=static)
    n = y.shape[0]
    scale = float(np.mean(hdiag)) / n
    q = y / hdiag
    Gq = G @ q
    loss = float(q @ Gq - 2.0 * q @ rhat) * scale
    # d loss / d q = (G + G^T) q - 2 rhat; the library uses 2 G q (G is symmetric up to the small
    # asymmetry of S), and so does this reference
    dy = (2.0 * (Gq - rhat) / hdiag * scale)[None, :]
    dWs, dbs = [None] * 3, [None] * 3
    for i in (2, 1, 0):
        if i < 2:
            dy = dy * (acts[i + 1] > 0.0)
        dx, dWs[i], dbs[i] = conv_grads(acts[i], W[i], dy, nb, nlev)
        dy = dx
    return loss, dWs, dbs
