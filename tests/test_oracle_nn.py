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


# ---- the stage after the two-level cycle ----

def _stage_problem():
    from oracle.problem import OracleProblem
    from synth import make_box

    prob = make_box(nx=6, ny=4, nlev=5, dx=5e3, dz=250.0, mg_levels=2, perturb=0.05, seed=3)
    orc = OracleProblem(prob)
    return prob, orc, orc.H.diagonal().copy(), nn.neighbour_table(prob.nx, prob.ny)


def test_identity_weights_give_the_identity():
    W, b = nn.identity_weights(4)
    x = np.random.default_rng(1).standard_normal(5 * 20)
    np.testing.assert_array_equal(nn.forward(x, W, b, nn.neighbour_table(5, 4), 5)[0], x)


def test_stage_with_identity_network_is_the_diagonal_coarse_correction():
    """N = identity turns the stage into d = P H_KK^-1 Gamma P^T r' (written out here directly)."""
    prob, orc, hd, nb = _stage_problem()
    S, P, gam = orc.hyb.S, orc.pc.P, orc.pc.gamma
    W, b = nn.identity_weights(16)
    rng = np.random.default_rng(4)
    accepted_any = False
    for _ in range(4):
        v = rng.standard_normal(S.shape[0])
        z = orc.pc(v)
        znew, acc = nn.learned_correction(v, z, S, P, gam, hd, W, b, nb, prob.nlev)
        rp = v - S @ z
        d = P @ ((gam * (P.T @ rp)) / hd)
        expect_acc = np.linalg.norm(rp - S @ d) < np.linalg.norm(rp)
        assert acc == expect_acc
        np.testing.assert_allclose(znew, z + d if acc else z, rtol=1e-12, atol=1e-12 * np.abs(z).max())
        accepted_any |= acc
    assert accepted_any  # the diagonal coarse correction helps on at least one of the vectors


def test_stage_is_positively_homogeneous():
    prob, orc, hd, nb = _stage_problem()
    S, P, gam = orc.hyb.S, orc.pc.P, orc.pc.gamma
    W, b = nn.init_weights(16, seed=5)
    rng = np.random.default_rng(6)
    v = rng.standard_normal(S.shape[0])
    z = orc.pc(v)
    z1, a1 = nn.learned_correction(v, z, S, P, gam, hd, W, b, nb, prob.nlev)
    for a in (3.7, 1e-5):
        za, aa = nn.learned_correction(a * v, a * z, S, P, gam, hd, W, b, nb, prob.nlev)
        assert aa == a1
        np.testing.assert_allclose(za, a * z1, rtol=1e-10, atol=1e-12 * a * np.abs(z1).max())


def test_stage_rejects_useless_and_harmful_corrections():
    prob, orc, hd, nb = _stage_problem()
    S, P, gam = orc.hyb.S, orc.pc.P, orc.pc.gamma
    v = np.random.default_rng(7).standard_normal(S.shape[0])
    z = orc.pc(v)
    W0 = [np.zeros((16, nn.NIN, nn.NT)), np.zeros((16, 16, nn.NT)), np.zeros((1, 16, nn.NT))]
    b0 = [np.zeros(16), np.zeros(16), np.zeros(1)]
    zn, acc = nn.learned_correction(v, z, S, P, gam, hd, W0, b0, nb, prob.nlev)
    assert np.array_equal(zn, z)  # a zero correction leaves z as it is, accepted or not
    W, b = nn.identity_weights(16)
    W[2] = W[2] * 1e8  # a correction far larger than the error
    zn, acc = nn.learned_correction(v, z, S, P, gam, hd, W, b, nb, prob.nlev)
    assert not acc and np.array_equal(zn, z)


def _symmetric_problem():
    """theta* constant (N = 0) makes S symmetric positive definite."""
    from oracle.problem import OracleProblem
    from synth import make_box

    prob = make_box(nx=6, ny=4, nlev=5, dx=5e3, dz=250.0, mg_levels=2, nbv=0.0, seed=3)
    orc = OracleProblem(prob)
    return prob, orc


def test_energy_loss_is_the_change_of_error_energy():
    """In the symmetric case the loss equals, up to its scale, the change of e'^T S e' when the
    correction P (s q) is added, with e' = S^-1 r' from a direct solve."""
    import scipy.sparse.linalg as spla

    prob, orc = _symmetric_problem()
    S, P, gam = orc.hyb.S.tocsc(), orc.pc.P, orc.pc.gamma
    assert abs(S - S.T).max() <= 1e-12 * abs(S).max()
    hd = orc.H.diagonal().copy()
    nb = nn.neighbour_table(prob.nx, prob.ny)
    W, b = nn.identity_weights(16)  # a correction of the size of the error (random weights are tiny)
    rng = np.random.default_rng(9)
    v = rng.standard_normal(S.shape[0])
    rp = v - S @ orc.pc(v)
    c = gam * (P.T @ rp)
    s = np.sqrt(np.mean(c * c))
    x, rhat = c / s, (P.T @ rp) / s
    loss = nn.energy_loss_and_grads(x, rhat, W, b, nb, prob.nlev, (P.T @ S @ P).tocsr(), hd)[0]
    e = spla.spsolve(S, rp)
    y = nn.forward(x, W, b, nb, prob.nlev)[0]
    d = P @ (s * y / hd)
    e_before, e_after = e @ (S @ e), (e - d) @ (S @ (e - d))
    scale = np.mean(hd) / prob.ncell / s**2
    # the change is a small difference of two energies: compare to the rounding of the energies
    assert abs(loss - (e_after - e_before) * scale) <= 1e-10 * (e_before + e_after) * scale
    assert abs(e_after - e_before) > 1e-4 * e_before  # the check is not vacuous


def test_energy_gradients_match_central_differences():
    prob, orc, hd, nb_ = _stage_problem()
    S, P = orc.hyb.S, orc.pc.P
    G = (P.T @ S @ P).tocsr()
    G = 0.5 * (G + G.T)  # the gradient assumes a symmetric G
    W, b = nn.init_weights(8, seed=11)
    rng = np.random.default_rng(12)
    for bi in b:
        bi[:] = rng.standard_normal(bi.shape) * 0.1
    x = rng.standard_normal(prob.ncell)
    rhat = rng.standard_normal(prob.ncell)
    f = lambda W_, b_: nn.energy_loss_and_grads(x, rhat, W_, b_, nb_, prob.nlev, G, hd)  # noqa: E731
    loss, dW, db = f(W, b)
    h = 1e-6
    for layer in range(3):
        for _ in range(4):
            idx = tuple(rng.integers(0, k) for k in W[layer].shape)
            Wp = [w.copy() for w in W]
            Wm = [w.copy() for w in W]
            Wp[layer][idx] += h
            Wm[layer][idx] -= h
            fd = (f(Wp, b)[0] - f(Wm, b)[0]) / (2 * h)
            assert abs(fd - dW[layer][idx]) <= 1e-6 * max(1.0, abs(fd)), (layer, idx, fd, dW[layer][idx])
        bp = [v.copy() for v in b]
        bm = [v.copy() for v in b]
        bp[layer][0] += h
        bm[layer][0] -= h
        fd = (f(W, bp)[0] - f(W, bm)[0]) / (2 * h)
        assert abs(fd - db[layer][0]) <= 1e-6 * max(1.0, abs(fd))


def test_neighbour_table_from_tables_on_the_box():
    from synth import make_box

    p = make_box(nx=5, ny=4, nlev=1, dx=1e3, dz=1e3, mg_levels=1)
    np.testing.assert_array_equal(nn.neighbour_table_from_tables(p.col_edge, p.edge_col, p.edge_lf),
                                  nn.neighbour_table(5, 4))


def test_neighbour_table_on_the_cubed_sphere():
    # edge neighbours share two corner points with the column, corner neighbours exactly one, and
    # the tap's direction agrees with the geometry: the neighbour's centre lies on the side of the
    # offset (dx, dy) in the column's frame; only the 3 columns at each of the 8 cube vertices lack
    # the corner neighbour there
    from synth import make_sphere

    p = make_sphere(6, 1, mg_levels=1)
    nb = nn.neighbour_table_from_tables(p.col_edge, p.edge_col, p.edge_lf)
    U = np.round(p.corners, 12)
    ncol = p.ncol
    pts = [set(map(tuple, U[:, :, c])) for c in range(ncol)]
    assert (nb < 0).sum() == 24
    cen = p.column_centres()
    ex = (U[1] + U[3] - U[0] - U[2])  # the frame's x and y directions at the column
    ey = (U[2] + U[3] - U[0] - U[1])
    for h, (dx, dy) in enumerate(nn.H_OFFSETS[1:], start=1):
        for c in range(ncol):
            n = nb[h, c]
            if n < 0:
                continue
            shared = len(pts[c] & pts[n])
            assert shared == (2 if h <= 4 else 1), (h, c, n)
            d = cen[:, n] - cen[:, c]
            assert dx * (d @ ex[:, c]) >= 0 and dy * (d @ ey[:, c]) >= 0
            if dx:
                assert dx * (d @ ex[:, c]) > 0
            if dy:
                assert dy * (d @ ey[:, c]) > 0


def test_gradients_with_missing_neighbours():
    from synth import make_sphere

    p = make_sphere(2, 4, mg_levels=1)
    nb = nn.neighbour_table_from_tables(p.col_edge, p.edge_col, p.edge_lf)
    assert (nb < 0).any()
    nlev, n = 4, p.ncell
    W, b = nn.init_weights(3, 5)
    rng = np.random.default_rng(6)
    x, t = rng.standard_normal(n), rng.standard_normal(n)
    loss, dW, db, dx = nn.loss_and_grads(x, t, W, b, nb, nlev)
    h = 1e-6
    for layer in range(3):
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in W[layer].shape)
            Wp = [w.copy() for w in W]
            Wm = [w.copy() for w in W]
            Wp[layer][idx] += h
            Wm[layer][idx] -= h
            fd = (nn.loss_and_grads(x, t, Wp, b, nb, nlev)[0] - nn.loss_and_grads(x, t, Wm, b, nb, nlev)[0]) / (2 * h)
            assert abs(fd - dW[layer][idx]) <= 1e-6 * max(1.0, abs(fd))
    for i in rng.integers(0, n, 10):
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        fd = (nn.loss_and_grads(xp, t, W, b, nb, nlev)[0] - nn.loss_and_grads(xm, t, W, b, nb, nlev)[0]) / (2 * h)
        assert abs(fd - dx[i]) <= 1e-6 * max(1.0, abs(fd))


def test_static_inputs():
    # log(h / dz) and the centre height over the lid's, from volumes and interface heights
    z = np.array([0.0, 10.0, 40.0, 100.0])
    ncol = 2
    dz = np.repeat(np.diff(z), ncol)
    vol = np.repeat([4e4, 9e4, 16e4], ncol) * dz  # h = 200, 300, 400
    st = nn.static_inputs(vol, z, ncol)
    np.testing.assert_allclose(st[0], np.log(np.repeat([200 / 10, 300 / 30, 400 / 60], ncol)), rtol=1e-14)
    np.testing.assert_allclose(st[1], np.repeat([5 / 100, 25 / 100, 70 / 100], ncol), rtol=1e-14)


def test_gradients_with_static_inputs():
    # the static channels enter the first layer like the residual channel (finite differences)
    nb, W, b, x, t = _setup()
    nlev = 6
    st = np.random.default_rng(9).standard_normal((2, x.shape[0]))
    loss, dW, db, _ = nn.loss_and_grads(x, t, W, b, nb, nlev, static=st)
    h = 1e-6
    rng = np.random.default_rng(4)
    for _ in range(6):
        idx = (rng.integers(0, W[0].shape[0]), rng.integers(1, 3), rng.integers(0, nn.NT))
        Wp = [w.copy() for w in W]
        Wm = [w.copy() for w in W]
        Wp[0][idx] += h
        Wm[0][idx] -= h
        fd = (nn.loss_and_grads(x, t, Wp, b, nb, nlev, static=st)[0]
              - nn.loss_and_grads(x, t, Wm, b, nb, nlev, static=st)[0]) / (2 * h)
        assert abs(fd - dW[0][idx]) <= 1e-6 * max(1.0, abs(fd))
    # a network reading only a static channel through its centre tap is the identity on it
    Wi, bi = nn.identity_weights(16)
    Wi[0][:, [0, 1], :] = Wi[0][:, [1, 0], :]  # route static channel 1 instead of the residual
    y, _ = nn.forward(x, Wi, bi, nb, nlev, static=st)
    np.testing.assert_allclose(y, st[0], atol=1e-14)
