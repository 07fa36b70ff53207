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


@pytest.mark.gpu
def test_network_forward_and_gradients_match_oracle(small):
    prob, s = small
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
    errs = []
    off = 0
    for name, shp in learned.layout():
        nn_ = int(np.prod(shp))
        errs.append(rel_max(g[off : off + nn_], gref[off : off + nn_]))
        off += nn_
    say(f"[nn] forward {err_y:.2e} loss {loss:.6e} vs {lref:.6e} grads {['%.1e' % e for e in errs]}")
    assert err_y <= 1e-5
    assert abs(loss - lref) <= 1e-5 * lref
    assert max(errs) <= 1e-4


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
def test_energy_loss_gradients_match_oracle(small):
    """The training loss of the stage (error energy after the correction) and its gradients against
    the oracle's, with G = P^T S P and the oracle's S (which the GPU's matches to 1e-12)."""
    prob, s = small
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
    errs, off = [], 0
    for name, shp in learned.layout():
        k = int(np.prod(shp))
        errs.append(rel_max(g[off : off + k], gref[off : off + k]))
        off += k
    say(f"[energy] loss {loss:.6e} vs {lref:.6e}; grads {['%.1e' % e for e in errs]}")
    assert abs(loss - lref) <= 1e-5 * abs(lref)
    assert max(errs) <= 1e-4


def _stage_reference(prob, orc, vec, v, round_act):
    """The stage with the network's BF16 weights, in FP64: with round_act = bf16_round the hidden
    activations are rounded to BF16 as the kernels store them; with None the network is the
    unrounded one.  Returns (z, accepted, z of the plain cycle)."""
    W, b = learned.unpack(vec)
    Wr = [onn.bf16_round(w) for w in W]
    z = orc.pc(v)
    zs, acc = onn.learned_correction(v, z, orc.pc.S, orc.pc.P, orc.pc.gamma, orc.H.diagonal(), Wr, b,
                                     onn.neighbour_table(prob.nx, prob.ny), prob.nlev, round_act=round_act,
                                     static=static_for(prob))
    return zs, acc, z


@pytest.mark.gpu
def test_precondition_with_learned_stage_matches_oracle(small):
    """hyb_precondition with the stage against the oracle's cycle + stage.  Against the unrounded
    FP64 network (BF16 weights): the kernels store hidden activations in BF16 (relative rounding
    2^-9 per value, through two hidden layers), so the correction may differ by 2^-6 of its own size
    (measured 2e-3 to 6e-3).  Against the network with BF16-rounded activations (the kernels'
    storage format): an exact identity network to 1e-6 (every product is exact in BF16 / FP32) and a
    random one to 1e-4 (where the FP32 accumulation on the GPU and the FP64 one in the oracle
    straddle a BF16 rounding boundary, a hidden activation differs by one BF16 ulp)."""
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
            zref, acc, z0 = _stage_reference(prob, orc, vec, v, onn.bf16_round)
            zex, acc_ex, _ = _stage_reference(prob, orc, vec, v, None)
            z = torch.empty(s.ntrace, dtype=torch.float64, device="cuda")
            p.learned = 1
            s.set_params(p)
            s.precondition(dev(v), z)
            p.learned = 0
            s.set_params(p)
            err = rel_max(host(z), zref)
            err_ex = rel_max(host(z), zex)
            corr = rel_max(zex, z0)  # the correction's size relative to the result
            say(f"[stage] {name} trial {trial}: accepted {acc}, error {err:.2e}; against the unrounded network "
                f"{err_ex:.2e} = {err_ex / max(corr, 1e-300):.1e} of the correction")
            assert acc == acc_ex
            assert err_ex <= 2.0**-6 * corr
            assert err <= (1e-6 if name == "identity" else 1e-4)


@pytest.mark.gpu
def test_learned_stage_trains_and_gains():
    """Train on the energy loss with pairs from the plain method on a 32x32x64 box (dx = 5 km,
    dz = 250 m), then compare FGMRES iterations to 1e-8 with and without the stage on held-out
    right-hand sides; every solve is checked with the oracle's S."""
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
    plain, with_nn, used = [], [], []
    for seed in (1000, 1001, 1002):
        r_ub, r_pi = make_rhs(prob, seed)
        b = rhs(seed)
        for flag, out in ((0, plain), (1, with_nn)):
            p = s.params
            p.learned = flag
            s.set_params(p)
            lam = torch.zeros_like(b)
            info = s.solve(b, lam, rtol=1e-8)
            ruc, rpc = cells_from_soa(r_ub, r_pi)
            B = orc.hyb.rhs(ruc, rpc)
            res = np.linalg.norm(B - orc.hyb.S @ host(lam)) / np.linalg.norm(B)
            assert info["status"] == 0 and res <= 1.01e-8
            out.append(info["iters"])
            if flag:
                used.append(info["iters"] - info["fallbacks"])
    p = s.params
    p.learned = 0
    s.set_params(p)
    say(f"[learned] held-out iterations: plain {plain}, with learned stage {with_nn} "
        f"(corrections kept {used})")
    assert sum(used) > 0
    assert sum(with_nn) < sum(plain)


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
    # a fresh context whose first network call is a training step (batch 3)
    s = make_solver(prob)
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
