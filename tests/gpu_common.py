"""Helpers shared by the GPU tests: move a synthetic problem onto the device and build a solver."""

from __future__ import annotations

import sys

import numpy as np

from paper_2210_11797_amd import HybSolver, Params, levels_of, solver_for  # noqa: F401


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def params_for(prob, **kw):
    base = dict(dt=prob.dt, tau_u=prob.tau_u, tau_rho=prob.tau_rho, tau_theta=prob.tau_theta, cp=prob.cp,
                rd=prob.rd, omega_rot=getattr(prob, "omega_rot", 0.0))
    base.update(kw)
    return Params(**base)


def make_solver(prob, **kw):
    s = solver_for(prob, params_for(prob, **kw))
    s.assemble_local(dev(prob.theta_w), dev(prob.exner_hat_w), dev(prob.exner_c), dev(prob.rho_c))
    s.condense()
    return s


def rel_max(a, ref):
    ref = np.asarray(ref)
    return float(np.abs(np.asarray(a) - ref).max() / max(np.abs(ref).max(), 1e-300))


def rel_norm(a, ref):
    ref = np.asarray(ref)
    return float(np.linalg.norm(np.asarray(a) - ref) / max(np.linalg.norm(ref), 1e-300))


def static_for(prob, orc=None):
    """The network's static input channels for a synthetic problem, computed by the oracle (cell
    volumes of its own cell matrices on the sphere, dx dy dz on the box)."""
    from oracle import nn as onn

    if getattr(prob, "geom", "box") == "shell":
        if orc is None:
            from oracle.problem import OracleProblem

            orc = OracleProblem(prob, with_mixed=False, with_precond=False)
        vol = orc.loc["m3"]
    else:
        vol = prob.dx * prob.dy * np.repeat(np.diff(prob.z), prob.ncol)
    return onn.static_inputs(vol, prob.z, prob.ncol)


def oracle_all_rows(spec, sols, tmpdir, timeout=900):
    """The oracle's all-rows residuals (oracle/allrows.py) of candidate solutions [(lam, u_b, pi)],
    computed in a separate process (a pool of forked CPU workers that never touch the GPU) for the
    synthetic problem ``spec`` and its right-hand side seed."""
    import json
    import os
    import subprocess

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    path = os.path.join(str(tmpdir), "candidates.npz")
    arrays = {"count": len(sols)}
    for i, (lam, ub, pi) in enumerate(sols):
        arrays.update({f"lam{i}": lam, f"ub{i}": ub, f"pi{i}": pi})
    np.savez(path, **arrays)
    workers = max(1, min(16, os.cpu_count() or 1))
    say(f"[oracle all rows] {spec} with {workers} worker processes")
    out = subprocess.run([sys.executable, "-m", "oracle.allrows", json.dumps(spec), path, str(workers)],
                         capture_output=True, text=True, cwd=root, timeout=timeout)
    if out.returncode != 0:
        raise RuntimeError(out.stderr[-3000:])
    return json.loads(out.stdout.strip().splitlines()[-1])
