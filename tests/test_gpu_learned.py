"""Learned coarse correction on the GPU: network passes and gradients against the FP64 oracle,
restriction, training, the solve with the stage, its fallback, and what it gains (GPU)."""

import numpy as np
import pytest

from gpu_common import dev, host, make_solver, rel_max, say, static_for
from oracle import nn as onn
from oracle.problem import OracleProblem, cells_from_soa
from paper_2210_11797_amd import learned
from synth import make_box, make_rhs


def _f32(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.fixture(scope="module")
def small():
    prob = make_box(nx=12, ny=10, nlev=9, dx=5e3, dz=250.0, mg_levels=2, perturb=0.05)
    s = make_solver(prob)
    return prob, s


# The training passes in BF16 (the default): every hidden activation and backpropagated field is
# rounded to BF16 once (unit roundoff u = 2^-9) and enters products accumulated in FP32.  The
# forward pass may then differ from the FP64 network by 2^-6 of its largest entry (about eight
# roundings in a row; measured 2e-3 to 5e-3).  A gradient is a sum over all cells of terms whose
# rounding errors do not cancel as the terms do, so its error is measured against the magnitude
# of its terms, the same backward pass run on absolute values (|activations|, |weights|, and |dy|
# widened by the forward error of y): within u of that magnitude per parameter group (measured
# 2e-6 to 4e-4).  The FP32 reference path (nn_fp32 = 1) keeps the oracle's 1e-5 / 1e-4 of the
# largest entry.
TOL = {1: dict(y=1e-5, loss=1e-5, grad=1e-4), 0: dict(y=2.0**-6, loss=2.0**-6, grad=2.0**-9)}


def _grad_magnitude(x, target, W, b, nb, nlev, st, G=None, hd=None):
    """Per parameter, the sum of the absolute values of the terms of the oracle's gradient (MSE
    against target, or with G and hd the energy loss against rhat = target): the backward pass on
    |activations| and |weights| from |dy| plus the bound 2 |G| |y|_abs / hd^2 (energy) or 2 |y|_abs
    (MSE) of the error that the forward pass passes into dy (|y|_abs: the last layer on absolute
    values).  Returned in the packed parameter layout."""
    y, acts = onn.forward(x, W, b, nb, nlev, static=st)
    n = y.shape[0]
    ya = onn.conv(np.abs(acts[2]), np.abs(W[2]), np.abs(b[2]), nb, nlev)[0]
    if G is not None:
        scale = float(np.mean(hd)) / n
        dya = (np.abs(2.0 * (G @ (y / hd) - target) / hd) + 2.0 * (abs(G) @ (ya / hd)) / hd) * scale
    else:
        dya = (2.0 / n) * (np.abs(y - target) + ya)
    dyA = dya[None, :]
    mW, mb = [None] * 3, [None] * 3
    for i in (2, 1, 0):
        if i < 2:
            dyA = dyA * (acts[i + 1] > 0.0)
        dyA, mW[i], mb[i] = onn.conv_grads(np.abs(acts[i]), np.abs(W[i]), dyA, nb, nlev)
    return learned.pack(mW, mb).astype(np.float64)


def _grad_errors(g, gref, mag, fp32):
    """Per parameter group: the largest error over the largest gradient entry (FP32 path) or over
    the largest magnitude of the terms (BF16 path)."""
    errs, off = [], 0
    for name, shp in learned.layout():
        k = int(np.prod(shp))
        d = np.abs(g[off : off + k] - gref[off : off + k]).max()
        errs.append(float(d / (np.abs(gref[off : off + k]).max() if fp32 else mag[off : off + k].max())))
        off += k
    return errs


def _set_fp32(s, fp32):
    p = s.params
    p.nn_fp32 = fp32
    s.set_params(p)


@pytest.mark.gpu
@pytest.mark.parametrize("fp32", [1, 0])
def test_network_forward_and_gradients_match_oracle(small, fp32):
    prob, s = small
    _set_fp32(s, fp32)
    rng = np.random.default_rng(0)
    vec = learned.init_params(16, seed=1)
    vec[16 * learned.NIN * 45 : 16 * learned.NIN * 45 + 16] = rng.standard_normal(16) * 0.1  # b1
    s.nn_set_weights(vec)
    x = rng.standard_normal((2, prob.ncell)).astype(np.float32)
    t = rng.standard_normal((2, prob.ncell)).astype(np.float32)
    W, b = learned.unpack(vec)
    Wr = [onn.bf16_round(w) for w in W]  # the kernels use BF16 weights, FP32 biases
    nb = onn.neighbour_table(prob.nx, prob.ny)
    import torch

    y = torch.empty((2, prob.ncell), dtype=torch.float32, device="cuda")
    s.nn_forward(_f32(x), y, 2)
    st = static_for(prob)
    yref = np.stack([onn.forward(x[i].astype(np.float64), Wr, b, nb, prob.nlev, static=st)[0] for i in range(2)])
    err_y = rel_max(host(y), yref)
    loss, g = s.nn_loss_grad(_f32(x), _f32(t), 2)
    # oracle: mean over both samples = average of the per-sample means
    refs = [onn.loss_and_grads(x[i].astype(np.float64), t[i].astype(np.float64), Wr, b, nb, prob.nlev, static=st)
            for i in range(2)]
    lref = 0.5 * (refs[0][0] + refs[1][0])
    gW = [0.5 * (refs[0][1][j] + refs[1][1][j]) for j in range(3)]
    gb = [0.5 * (refs[0][2][j] + refs[1][2][j]) for j in range(3)]
    gref = learned.pack(gW, gb).astype(np.float64)
    mag = 0.5 * sum(_grad_magnitude(x[i].astype(np.float64), t[i].astype(np.float64), Wr, b, nb, prob.nlev, st)
                    for i in range(2))
    errs = _grad_errors(g, gref, mag, fp32)
    say(f"[nn fp32={fp32}] forward {err_y:.2e} loss {loss:.6e} vs {lref:.6e} grads {['%.1e' % e for e in errs]}")
    _set_fp32(s, 0)
    assert err_y <= TOL[fp32]["y"]
    assert abs(loss - lref) <= TOL[fp32]["loss"] * lref
    assert max(errs) <= TOL[fp32]["grad"]


def _sparse_exact_net(rng):
    """Weights of +-1 (sparse) that keep every activation and backpropagated field of the exact-case
    inputs below 2^8 in magnitude with few significant bits, so that BF16 stores them exactly."""
    def sparse(shape, dens):
        return (rng.random(shape) < dens) * rng.choice([-1.0, 1.0], shape)

    W = [sparse((16, learned.NIN, 45), 0.08), sparse((16, 16, 45), 0.03), sparse((1, 16, 45), 0.05)]
    W[0][:, 1:, :] = 0.0  # the static channels (not BF16 numbers) enter only the first layer's gradient
    return W, [np.zeros(16), np.zeros(16), np.zeros(1)]


@pytest.mark.gpu
@pytest.mark.parametrize("mesh", ["box8x6x5", "sphere_c4x5"])
def test_bf16_training_exact_case(mesh):
    """The BF16 matrix-core training passes against the FP64 oracle where BF16 is exact: +-1 weights,
    inputs in {-1, 0, 1} and targets y + {-2..2}, so every stored activation and backpropagated
    field is a BF16 number (checked on the oracle's values).  The forward pass must then be exact
    and the gradients exact up to the FP32 rounding of sums and of the final 1 / (samples x cells)
    (1e-6 of the largest entry), except the first layer's static-channel weights, whose inputs are
    rounded to BF16 (2^-7).  On the cubed sphere this covers the transposed convolution through the
    columns read twice through one tap next to cube edges."""
    import torch

    from synth import make_sphere

    if mesh.startswith("sphere"):
        prob = make_sphere(4, 5, mg_levels=2, perturb=0.05)
        nb = onn.neighbour_table_from_tables(prob.col_edge, prob.edge_col, prob.edge_lf)
    else:
        prob = make_box(nx=8, ny=6, nlev=5, dx=5e3, dz=250.0, mg_levels=2, perturb=0.05, seed=5)
        nb = onn.neighbour_table(prob.nx, prob.ny)
    s = make_solver(prob)
    st = static_for(prob)
    rng = np.random.default_rng(3)
    W, b = _sparse_exact_net(rng)
    vec = learned.pack(W, b)
    x = rng.integers(-1, 2, (2, prob.ncell)).astype(np.float64)
    fw = [onn.forward(x[i], W, b, nb, prob.nlev, static=st) for i in range(2)]
    t = np.stack([np.round(y) + rng.integers(-2, 3, prob.ncell) for y, _ in fw])
    refs = [onn.loss_and_grads(x[i], t[i], W, b, nb, prob.nlev, static=st) for i in range(2)]
    for _, acts in fw:
        for a in acts[1:3]:
            assert np.array_equal(onn.bf16_round(a), a)  # the case is exact in BF16
    gref = learned.pack([0.5 * (refs[0][1][j] + refs[1][1][j]) for j in range(3)],
                        [0.5 * (refs[0][2][j] + refs[1][2][j]) for j in range(3)]).astype(np.float64)
    s.nn_set_weights(vec)
    y = torch.empty((2, prob.ncell), dtype=torch.float32, device="cuda")
    s.nn_forward(_f32(x), y, 2)
    err_y = float(np.abs(host(y) - np.stack([f[0] for f in fw])).max())
    loss, g = s.nn_loss_grad(_f32(x), _f32(t), 2)
    lref = 0.5 * (refs[0][0] + refs[1][0])
    errs, off = {}, 0
    for name, shp in learned.layout():
        k = int(np.prod(shp))
        gg, rr = g[off : off + k].reshape(shp), gref[off : off + k].reshape(shp)
        scale = np.abs(rr).max()
        if name == "W1":
            errs["W1 x"] = float(np.abs(gg[:, :1] - rr[:, :1]).max() / scale)
            errs["W1 static"] = float(np.abs(gg[:, 1:] - rr[:, 1:]).max() / scale)
        else:
            errs[name] = float(np.abs(gg - rr).max() / scale)
        off += k
    say(f"[bf16 exact {mesh}] forward max diff {err_y:.1e}, loss {loss:.6e} vs {lref:.6e}, "
        + " ".join(f"{a} {e:.1e}" for a, e in errs.items()))
    s.close()
    assert err_y == 0.0
    assert abs(loss - lref) <= 1e-6 * lref
    assert errs.pop("W1 static") <= 2.0**-7
    assert max(errs.values()) <= 1e-6


@pytest.mark.gpu
def test_restriction_modes(small):
    prob, s = small
    import torch

    orc = OracleProblem(prob)
    r = np.random.default_rng(2).standard_normal(orc.mesh.ntrace)
    c = torch.empty(prob.ncell, dtype=torch.float64, device="cuda")
    s.restrict(dev(r), c, 0)
    P, S, H = orc.pc.P, orc.pc.S, orc.pc.mg.H[0]
    # Gamma = (H 1) / (P^T S P 1): both sums cancel (row sums of H and S are small against their
    # entries), so the rounding of either side is eps times the cancellation ratio sum|a| / |sum a|
    one = np.ones(prob.ncell)
    ratio = np.max((abs(H) @ one) / abs(H @ one)) + np.max(
        (abs(P).T @ (abs(S) @ (abs(P) @ one))) / abs(P.T @ (S @ (P @ one))))
    tol = 4 * np.finfo(float).eps * ratio
    err = rel_max(host(c), orc.pc.gamma * (P.T @ r))
    say(f"[restrict] Gamma P^T r: {err:.2e} (tol {tol:.2e}, cancellation ratio {ratio:.2e})")
    assert err <= tol
    s.restrict(dev(r), c, 1)
    avg = (P.T @ r) / (P.T @ np.ones(orc.mesh.ntrace))
    assert rel_max(host(c), avg) <= 1e-12
    s.restrict(dev(r), c, 2)
    assert rel_max(host(c), orc.H.diagonal() * avg) <= 1e-12
    s.restrict(dev(r), c, 3)
    assert rel_max(host(c), P.T @ r) <= 1e-12


@pytest.mark.gpu
@pytest.mark.parametrize("fp32", [1, 0])
def test_energy_loss_gradients_match_oracle(small, fp32):
    """The training loss of the stage (error energy after the correction) and its gradients against
    the oracle's, with G = P^T S P and the oracle's S (which the GPU's matches to 1e-12), in the FP32
    reference path and the BF16 one (tolerances in TOL)."""
    prob, s = small
    _set_fp32(s, fp32)
    orc = OracleProblem(prob)
    P, S = orc.pc.P, orc.pc.S
    G = (P.T @ S @ P).tocsr()
    hd = orc.H.diagonal().copy()
    rng = np.random.default_rng(13)
    vec = learned.init_params(16, seed=14)
    vec[16 * learned.NIN * 45 : 16 * learned.NIN * 45 + 16] = rng.standard_normal(16) * 0.1
    vec[-1] = 0.3
    s.nn_set_weights(vec)
    x = rng.standard_normal((2, prob.ncell)).astype(np.float32)
    rhat = rng.standard_normal((2, prob.ncell))
    loss, g = s.nn_energy_grad(_f32(x), dev(rhat), 2)
    W, b = learned.unpack(vec)
    Wr = [onn.bf16_round(w) for w in W]
    nb = onn.neighbour_table(prob.nx, prob.ny)
    st = static_for(prob)
    refs = [onn.energy_loss_and_grads(x[i].astype(np.float64), rhat[i], Wr, b, nb, prob.nlev, G, hd, static=st)
            for i in range(2)]
    lref = 0.5 * (refs[0][0] + refs[1][0])
    gref = learned.pack([0.5 * (refs[0][1][j] + refs[1][1][j]) for j in range(3)],
                        [0.5 * (refs[0][2][j] + refs[1][2][j]) for j in range(3)]).astype(np.float64)
    mag = 0.5 * sum(_grad_magnitude(x[i].astype(np.float64), rhat[i], Wr, b, nb, prob.nlev, st, G, hd)
                    for i in range(2))
    errs = _grad_errors(g, gref, mag, fp32)
    say(f"[energy fp32={fp32}] loss {loss:.6e} vs {lref:.6e}; grads {['%.1e' % e for e in errs]}")
    _set_fp32(s, 0)
    assert abs(loss - lref) <= TOL[fp32]["loss"] * abs(lref)
    assert max(errs) <= TOL[fp32]["grad"]


def _stage_reference(prob, orc, vec, v):
    """The stage with the network's BF16 weights, in FP64 (the oracle's unrounded network).
    Returns (z, accepted, z of the plain cycle)."""
    W, b = learned.unpack(vec)
    Wr = [onn.bf16_round(w) for w in W]
    z = orc.pc(v)
    zs, acc = onn.learned_correction(v, z, orc.pc.S, orc.pc.P, orc.pc.gamma, orc.H.diagonal(), Wr, b,
                                     onn.neighbour_table(prob.nx, prob.ny), prob.nlev, static=static_for(prob))
    return zs, acc, z


# the stage's BF16 hidden activations (2^-9 per stored value) move its correction by at most this
# fraction of the correction's largest entry: the identity network rounds only its input (its
# products are exact; measured 2.3e-3 to 2.9e-3, the largest error and the largest correction
# falling on different facets), a random one rounds two hidden layers that feed 720 and 11520
# products per cell (measured 4.2e-3 to 5.2e-3)
STAGE_TOL = {"identity": 2.0**-7, "random": 2.0**-6}


@pytest.mark.gpu
def test_precondition_with_learned_stage_matches_oracle(small):
    """hyb_precondition with the stage against the oracle's cycle + stage with the unrounded FP64
    network (BF16 weights): the same acceptance decision, and the correction within STAGE_TOL of its
    size (measured 2e-3 to 6e-3 for the random network)."""
    prob, s = small
    import torch

    orc = OracleProblem(prob)
    Wi, bi = onn.identity_weights(16)
    nets = {"identity": learned.pack(Wi, bi), "random": learned.init_params(16, seed=9)}
    rng = np.random.default_rng(10)
    p = s.params
    for name, vec in nets.items():
        s.nn_set_weights(vec)
        for trial in range(3):
            v = rng.standard_normal(orc.mesh.ntrace)
            zex, acc_ex, z0 = _stage_reference(prob, orc, vec, v)
            z = torch.empty(s.ntrace, dtype=torch.float64, device="cuda")
            p.learned = 1
            s.set_params(p)
            s.precondition(dev(v), z)
            p.learned = 0
            s.set_params(p)
            err_ex = rel_max(host(z), zex)
            corr = rel_max(zex, z0)  # the correction's size relative to the result
            say(f"[stage] {name} trial {trial}: accepted {acc_ex}; against the unrounded network "
                f"{err_ex:.2e} = {err_ex / max(corr, 1e-300):.1e} of the correction")
            assert acc_ex and rel_max(host(z), z0) > 0.5 * corr  # the correction was applied
            assert err_ex <= STAGE_TOL[name] * corr


@pytest.mark.gpu
def test_learned_stage_trains_and_gains():
    """Train on the energy loss with pairs from the plain method on a 32x32x64 box (dx = 5 km,
    dz = 250 m), then compare FGMRES to 1e-8 with and without the stage on held-out right-hand
    sides: fewer iterations with the stage (every solve checked with the oracle's S), and the time
    criterion -- the time per solve with the stage is what its cost model predicts, iterations x
    (a plain iteration + a stage call - the trace matvec the stage's S application supplies) within
    25 %, so a net gain in time needs (plain iterations / learned iterations) > 1 + (stage - matvec)
    / iteration; the test reports that ratio and the two times (the measured outcome at the
    benchmark sizes is recorded with the benchmark)."""
    import time

    import torch

    prob = make_box(nx=32, ny=32, nlev=64, dx=5e3, dz=250.0, dt=600.0, mg_levels=4)
    s = make_solver(prob)
    s.nn_set_weights(learned.init_params(16, seed=0))

    def rhs(seed):
        r_ub, r_pi = make_rhs(prob, seed)
        b = torch.empty(s.ntrace, dtype=torch.float64, device="cuda")
        s.condense(dev(r_ub), dev(r_pi), b)
        return b

    X, R = learned.generate_pairs(s, [rhs(10000 + i) for i in range(48)], steps=8)
    say(f"[learned] {X.shape[0]} pairs")
    hist = learned.train(s, X, R, steps=1500, batch=8, lr=2e-3, log=say)
    assert np.mean(hist[-50:]) < np.mean(hist[:5])  # the energy loss starts near 0 and goes negative
    orc = OracleProblem(prob, with_precond=False)
    plain, with_nn, used, secs = [], [], [], {0: 0.0, 1: 0.0}
    seeds = (1000, 1001, 1002)
    for flag, out in ((0, plain), (1, with_nn)):
        p = s.params
        p.learned = flag
        s.set_params(p)
        s.solve(rhs(seeds[0]), torch.zeros(s.ntrace, dtype=torch.float64, device="cuda"), rtol=1e-8)  # warm-up
        for seed in seeds:
            r_ub, r_pi = make_rhs(prob, seed)
            b = rhs(seed)
            lam = torch.zeros_like(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = s.solve(b, lam, rtol=1e-8)
            torch.cuda.synchronize()
            secs[flag] += time.perf_counter() - t0
            ruc, rpc = cells_from_soa(r_ub, r_pi)
            B = orc.hyb.rhs(ruc, rpc)
            res = np.linalg.norm(B - orc.hyb.S @ host(lam)) / np.linalg.norm(B)
            assert info["status"] == 0 and res <= 1.01e-8
            out.append(info["iters"])
            if flag:
                used.append(info["iters"] - info["fallbacks"])
    # the cost model's parts, timed with events around each family
    b = rhs(seeds[0])
    costs = {}
    for fam, flag in (("nn", 1), ("trace_apply", 0)):
        p = s.params
        p.learned = flag
        s.set_params(p)
        s.profile_family(fam)
        s.solve(b, torch.zeros_like(b), rtol=1e-8)
        n, ms = s.profile_read(fam)
        s.profile(False)
        costs[fam] = ms / max(n, 1) / 1e3
    p = s.params
    p.learned = 0
    s.set_params(p)
    t_iter = secs[0] / sum(plain)
    model = sum(with_nn) * (t_iter + costs["nn"] - costs["trace_apply"])
    breakeven = 1.0 + (costs["nn"] - costs["trace_apply"]) / t_iter
    say(f"[learned] held-out iterations: plain {plain}, with learned stage {with_nn} (corrections kept {used}); "
        f"time {secs[0] * 1e3:.1f} ms plain, {secs[1] * 1e3:.1f} ms with the stage (model {model * 1e3:.1f} ms); "
        f"stage {costs['nn'] * 1e3:.2f} ms per call, iteration {t_iter * 1e3:.2f} ms, matvec "
        f"{costs['trace_apply'] * 1e3:.2f} ms: a time gain needs an iteration ratio above {breakeven:.2f}, "
        f"measured {sum(plain) / sum(with_nn):.2f}")
    assert sum(used) > 0
    assert sum(with_nn) < sum(plain)
    assert abs(secs[1] - model) <= 0.25 * model
    s.close()


@pytest.mark.gpu
def test_learned_stage_falls_back_on_overflow(small):
    prob, s = small
    import torch

    vec = learned.init_params(16, seed=3)
    # layer 1: +1e30 on even and -1e30 on odd channels, so that some channel is positive wherever
    # the input's 3x3x5 box sum is nonzero; layer 2 (all 1e30) then overflows to inf, and layer 3
    # (mixed signs) gives inf or NaN.  (All-positive weights would give an exactly zero, finite
    # output for inputs whose box sums are all negative.)
    vec[: 16 * learned.NIN * 45] = np.repeat(np.where(np.arange(16) % 2 == 0, 1e30, -1e30), learned.NIN * 45)
    vec[16 * learned.NIN * 45 + 16 : 16 * learned.NIN * 45 + 16 + 16 * 16 * 45] = 1e30
    s.nn_set_weights(vec)
    p = s.params
    p.learned = 1
    s.set_params(p)
    r_ub, r_pi = make_rhs(prob, 3)
    b = torch.empty(s.ntrace, dtype=torch.float64, device="cuda")
    s.condense(dev(r_ub), dev(r_pi), b)
    lam = torch.zeros_like(b)
    info = s.solve(b, lam, rtol=1e-8)
    p.learned = 0
    s.set_params(p)
    say(f"[learned] overflow weights: iters {info['iters']} fallbacks {info['fallbacks']}")
    assert info["status"] == 0 and info["fallbacks"] == info["iters"]


@pytest.mark.gpu
def test_training_resumes_from_saved_adam_state(small, tmp_path):
    """Training saved with its Adam state (learned.save) and resumed in a fresh context
    (learned.resume) continues exactly as training without a break (bitwise: the passes are
    deterministic); a NaN network output, forced from the host, falls back at every iteration."""
    prob, s = small
    rng = np.random.default_rng(31)
    x = _f32(rng.standard_normal((3, prob.ncell)))
    rhat = dev(rng.standard_normal((3, prob.ncell)))
    vec = learned.init_params(16, seed=5)
    s.nn_set_weights(vec)
    for _ in range(4):
        s.nn_energy_train_step(x, rhat, 3, 1e-3)
    w4 = s.nn_get_weights()
    s.nn_set_weights(vec)
    for _ in range(2):
        s.nn_energy_train_step(x, rhat, 3, 1e-3)
    path = str(tmp_path / "stage.npz")
    learned.save(path, s.nn_get_weights(), {"steps": 2}, state=s.nn_get_state())
    s2 = make_solver(prob)
    meta = learned.resume(s2, path)
    for _ in range(2):
        s2.nn_energy_train_step(x, rhat, 3, 1e-3)
    w22 = s2.nn_get_weights()
    say(f"[resume] after {meta['steps']} + 2 steps: max difference {np.abs(w22 - w4).max():.1e}")
    assert np.array_equal(w22, w4)
    import torch

    from paper_2210_11797_amd import HYB_DEBUG_NAN_STAGE

    p = s2.params
    p.learned, p.debug = 1, HYB_DEBUG_NAN_STAGE
    s2.set_params(p)
    r_ub, r_pi = make_rhs(prob, 3)
    b = torch.empty(s2.ntrace, dtype=torch.float64, device="cuda")
    s2.condense(dev(r_ub), dev(r_pi), b)
    info = s2.solve(b, torch.zeros_like(b), rtol=1e-8)
    say(f"[resume] NaN stage output: iters {info['iters']} fallbacks {info['fallbacks']}")
    assert info["status"] == 0 and info["fallbacks"] == info["iters"]
    s2.close()
    s.nn_set_weights(vec)


@pytest.mark.gpu
def test_call_orders_that_once_met_unallocated_buffers():
    """Regression test of two call orders whose buffers were once used before allocation (found
    on the CPU stand-in, fixed): a training step as the first network call of a fresh context, and
    the FP32 preconditioner (mixed form, with and without the stage) before any solve.  The
    results are checked against the oracle's formulas and the FP64 preconditioner."""
    import torch

    prob = make_box(nx=12, ny=10, nlev=9, dx=5e3, dz=250.0, mg_levels=2, perturb=0.05, seed=3)
    rng = np.random.default_rng(21)
    nb = onn.neighbour_table(prob.nx, prob.ny)
    st = static_for(prob)
    # a fresh context whose first network call is a training step (batch 3; the FP32 reference
    # passes, so that the loss meets the oracle's to 1e-5)
    s = make_solver(prob, nn_fp32=1)
    vec = learned.init_params(16, seed=4)
    s.nn_set_weights(vec)
    x = rng.standard_normal((3, prob.ncell)).astype(np.float32)
    t = rng.standard_normal((3, prob.ncell)).astype(np.float32)
    loss = s.nn_train_step(_f32(x), _f32(t), 3, 1e-3)
    W, b = learned.unpack(vec)
    Wr = [onn.bf16_round(w) for w in W]
    lref = np.mean([onn.loss_and_grads(x[i].astype(np.float64), t[i].astype(np.float64), Wr, b, nb, prob.nlev,
                                       static=st)[0] for i in range(3)])
    say(f"[call order] first call a training step: loss {loss:.6e} vs oracle {lref:.6e}")
    assert abs(loss - lref) <= 1e-5 * abs(lref)
    s.close()
    # fresh contexts in the mixed form: the preconditioner before any solve, against FP64
    s64 = make_solver(prob)
    v = rng.standard_normal(s64.ntrace)
    z64 = torch.empty(s64.ntrace, dtype=torch.float64, device="cuda")
    s64.precondition(dev(v), z64)
    for learned_on in (0, 1):
        sm = make_solver(prob, precision=1, learned=learned_on)
        if learned_on:
            sm.nn_set_weights(vec)
        zm = torch.empty(sm.ntrace, dtype=torch.float64, device="cuda")
        sm.precondition(dev(v), zm)
        err = rel_max(host(zm), host(z64))
        say(f"[call order] FP32 preconditioner before any solve (stage {learned_on}): {err:.2e} from FP64")
        assert np.all(np.isfinite(host(zm)))
        if not learned_on:
            assert err <= 1e-5
        sm.close()
    s64.close()
