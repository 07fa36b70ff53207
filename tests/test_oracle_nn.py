"""Pins of the oracle's learned-correction network (CPU only)."""

import numpy as np

from oracle import nn


def _setup(nx=5, ny=4, nlev=6, ch=3, seed=0):
    nb = nn.neighbour_table(nx, ny)
    W, b = nn.init_weights(ch, seed)
    rng = np.random.default_rng(seed + 1)
    for bi in b:
        bi[:] = rng.standard_normal(bi.shape) * 0.1
    x = rng.standard_normal(nlev * nx * ny)
    t = rng.standard_normal(nlev * nx * ny)
    return nb, W, b, x, t


def test_gradients_match_central_differences():
    nb, W, b, x, t = _setup()
    nlev = 6
    loss, dW, db, dx = nn.loss_and_grads(x, t, W, b, nb, nlev)
    rng = np.random.default_rng(3)
    h = 1e-6
    for layer in range(3):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in W[layer].shape)
            Wp = [w.copy() for w in W]
            Wm = [w.copy() for w in W]
            Wp[layer][idx] += h
            Wm[layer][idx] -= h
            fd = (nn.loss_and_grads(x, t, Wp, b, nb, nlev)[0] - nn.loss_and_grads(x, t, Wm, b, nb, nlev)[0]) / (2 * h)
            assert abs(fd - dW[layer][idx]) <= 1e-6 * max(1.0, abs(fd)), (layer, idx, fd, dW[layer][idx])
        j = rng.integers(0, b[layer].shape[0])
        bp = [v.copy() for v in b]
        bm = [v.copy() for v in b]
        bp[layer][j] += h
        bm[layer][j] -= h
        fd = (nn.loss_and_grads(x, t, W, bp, nb, nlev)[0] - nn.loss_and_grads(x, t, W, bm, nb, nlev)[0]) / (2 * h)
        assert abs(fd - db[layer][j]) <= 1e-6 * max(1.0, abs(fd))
    for i in rng.integers(0, x.shape[0], 8):
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        fd = (nn.loss_and_grads(xp, t, W, b, nb, nlev)[0] - nn.loss_and_grads(xm, t, W, b, nb, nlev)[0]) / (2 * h)
        assert abs(fd - dx[i]) <= 1e-6 * max(1.0, abs(fd))


def test_translation_equivariance_on_the_periodic_box():
    nx, ny, nlev = 6, 5, 4
    nb, W, b, x, _ = _setup(nx, ny, nlev)
    y, _ = nn.forward(x, W, b, nb, nlev)
    xs = np.roll(x.reshape(nlev, ny, nx), shift=(1, 2), axis=(2, 1)).ravel()
    ys, _ = nn.forward(xs, W, b, nb, nlev)
    np.testing.assert_allclose(ys, np.roll(y.reshape(nlev, ny, nx), shift=(1, 2), axis=(2, 1)).ravel(), atol=1e-12)


def test_one_hot_tap_is_a_shift():
    nx, ny, nlev = 5, 4, 7
    nb = nn.neighbour_table(nx, ny)
    x = np.random.default_rng(0).standard_normal(nlev * nx * ny)
    for h, v in ((0, 2), (2, 0), (7, 4), (4, 3)):
        W = np.zeros((1, 1, nn.NT))
        W[0, 0, h * nn.NV + v] = 1.0
        y = nn.conv(x[None, :], W, np.zeros(1), nb, nlev)[0].reshape(nlev, ny, nx)
        dxo, dyo = nn.H_OFFSETS[h]
        dk = v - 2
        xr = x.reshape(nlev, ny, nx)
        for k in range(nlev):
            src = k + dk
            expect = np.zeros((ny, nx)) if not (0 <= src < nlev) else np.roll(xr[src], shift=(-dyo, -dxo), axis=(0, 1))
            np.testing.assert_array_equal(y[k], expect)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2.0**-8, 1.0 + 3 * 2.0**-9, -3.14159, 1e-30])
    r = nn.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0  # tie rounds to even mantissa
    assert r[2] == 1.0 + 2.0**-7
    assert abs(r[3] + 3.14159) <= 2.0**-8 * 4
    assert np.all(np.abs(r - vals) <= np.abs(vals) * 2.0**-8)
