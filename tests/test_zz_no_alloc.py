"""hyb_solve_noalloc, the solve that allocates nothing (its reduction scratch is a static device
array), against hyb_solve through the C ABI (GPU): the same kernels in the same order give the
same iterate bit for bit.  Two calls in a row on one device share the array; the second has a
smaller input (another, smaller mesh), so it reads back only what it wrote itself."""

import numpy as np
import pytest

from gpu_common import dev, host, make_solver, params_for, say
from synth import make_box, make_rhs


def _solve_both(prob, seed, **kw):
    import torch

    s = make_solver(prob, **kw)
    r_ub, r_pi = make_rhs(prob, seed)
    b = torch.empty(s.ntrace, dtype=torch.float64, device="cuda")
    s.condense(dev(r_ub), dev(r_pi), b)
    lam_ref = torch.zeros_like(b)
    info_ref = s.solve(b, lam_ref, rtol=1e-10, maxit=200)
    lam = torch.zeros_like(b)
    info = s.solve(b, lam, rtol=1e-10, maxit=200, noalloc=True)
    torch.cuda.synchronize()
    return s, b, host(lam_ref), info_ref, host(lam), info


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_solve_matches_solve(precision):
    big = make_box(nx=16, ny=16, nlev=8, dx=10e3, dz=1250.0, mg_levels=4, perturb=0.05)
    small = make_box(nx=6, ny=4, nlev=3, dx=10e3, dz=1000.0, mg_levels=2, perturb=0.1, seed=2)
    for name, prob, seed in (("16x16x8", big, 0), ("6x4x3", small, 1)):
        s, b, lam_ref, info_ref, lam, info = _solve_both(prob, seed, precision=precision)
        diff = float(np.abs(lam - lam_ref).max() / np.abs(lam_ref).max())
        say(f"[noalloc] {name} precision {precision}: {info['iters']} / {info_ref['iters']} iterations, "
            f"residual {info['rel_res']:.2e} / {info_ref['rel_res']:.2e}, max difference {diff:.1e}")
        assert info["status"] == 0 and info_ref["status"] == 0
        assert info["iters"] == info_ref["iters"]
        assert info["history"] == info_ref["history"]
        assert diff == 0.0
        # the context's own reduction buffers are intact: hyb_solve still gives the same result
        import torch

        lam2 = torch.zeros_like(b)
        info2 = s.solve(b, lam2, rtol=1e-10, maxit=200)
        assert info2["iters"] == info_ref["iters"] and np.array_equal(host(lam2), lam_ref)
        s.close()


@pytest.mark.gpu
def test_noalloc_solve_rejects_what_it_cannot_do():
    import torch

    prob = make_box(nx=6, ny=4, nlev=3, dx=10e3, dz=1000.0, mg_levels=2, seed=2)
    s = make_solver(prob)
    b = dev(np.random.default_rng(3).standard_normal(s.ntrace))
    lam = torch.zeros_like(b)
    s.set_params(params_for(prob, restart=62))  # its reduction partials exceed the 2 MiB array
    with pytest.raises(RuntimeError, match="static scratch holds"):
        s.solve(b, lam, rtol=1e-8, noalloc=True)
    s.set_params(params_for(prob, restart=61))
    info = s.solve(b, lam, rtol=1e-8, noalloc=True)
    assert info["status"] == 0
    s.set_params(params_for(prob))
    s.profile(True)
    with pytest.raises(RuntimeError, match="profiling"):
        s.solve(b, lam, rtol=1e-8, noalloc=True)
    s.profile(False)
    s.close()
