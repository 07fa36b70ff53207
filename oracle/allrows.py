"""Residuals of a candidate solution over every row, for meshes too large for the assembled
operators (test infrastructure).

The cell matrices are built a chunk of cells at a time (``local.local_matrices`` or
``local.shell_local_matrices`` restricted to the chunk), and every cell adds its share to the rows
of its facets:

* the trace system (Sec. 2.4): B_lambda = sum_K C_K^T [A_K^-1 R_K]_u and S lambda =
  sum_K C_K^T [A_K^-1 K_K lambda_K]_u, so the relative residual ||B - S lambda|| / ||B|| is the
  one the solver stops on, now over all rows;
* the recovered velocity's continuity: the two outward fluxes of every interior facet sum to zero
  for the exact solution (C^T X = B - S lambda, Sec. 2.4);
* the 2x2 system of Sec. 2.2 at (u, Pi): every interior facet's velocity taken as the mean of its two
  cells' globally oriented fluxes, the relative residual ||R - M x|| / ||R|| and the componentwise
  backward error max_i |R - M x|_i / (|M| |x| + |R|)_i (scale invariant per row: the rows of this
  system differ in scale by many orders of magnitude).  The facet term of g is left out, so theta* must be single
  valued on facets (horizontally homogeneous reference states).

``chunk_contributions`` is the work of one chunk (independent of the others, so a caller may run
chunks in parallel processes); ``all_rows`` sums them.  Parity: these are the plain definitions of
the quantities, evaluated with the oracle's own cell matrices.
"""

from __future__ import annotations

import numpy as np

from .hybrid import cell_rhs, cell_trace_operator


def chunk_contributions(cell_matrices, cell_faces, cell_sign, cells, r_ub_cells, r_pi_cells, cands):
    """Per-cell shares for ``cells``: B (n, 6) and, for every candidate (lam, u_b, pi, u_glob) in
    ``cands``, S lambda (n, 6), the 2x2 velocity rows M x (n, 6) with |M| |x|, and the pressure-row
    residual with its scale (n,)."""
    loc = cell_matrices(cells)
    faces, sgn = cell_faces[cells], cell_sign[cells]
    Sc = cell_trace_operator(loc)
    A = loc["A"]
    out = dict(faces=faces, b=cell_rhs(loc, r_ub_cells[cells], r_pi_cells[cells]), cands=[])
    for lam, u_b, pi, u_glob in cands:
        x = np.concatenate([sgn * u_glob[faces], pi[cells, None]], axis=1)  # outward fluxes and Pi
        ax = np.einsum("cij,cj->ci", A, x)
        aax = np.einsum("cij,cj->ci", np.abs(A), np.abs(x))
        # |A_K| |x - X_K|: the cell's own fluxes X_K satisfy its equations, so the 2x2 residual of a
        # row is what replacing them by the facet means changes, bounded by this
        adev = np.einsum("cij,cj->ci", np.abs(A[:, :, :6]), np.abs(x[:, :6] - u_b[cells]))
        out["cands"].append(dict(sl=np.einsum("cfg,cg->cf", Sc, lam[faces]), mu=sgn * ax[:, :6], mu_abs=aax[:, :6],
                                 mu_dev=adev[:, :6], rp=r_pi_cells[cells] - ax[:, 6],
                                 rp_abs=aax[:, 6] + np.abs(r_pi_cells[cells]), rp_dev=adev[:, 6]))
    return out


def all_rows(cell_matrices, mesh, r_ub_cells, r_pi_cells, solutions, chunk=32768, map_fn=map):
    """For every candidate (lam, u_b, pi) in ``solutions`` (u_b (ncell, 6) outward fluxes, pi
    (ncell,)) returns dict(trace_res = ||B - S lambda|| / ||B||, defect_norm = ||C^T X|| / ||B||
    (the outward fluxes of every facet summed over its cells), defect = its largest entry / ||B||,
    mixed_res = ||R - M x|| / ||R|| and mixed_berr of the 2x2 system, and mixed_berr_bound: the
    backward error that the continuity defect alone can cause, max_i (|M| |x - X|)_i / (|M| |x| + |R|)_i
    with X the cells' own recovered fluxes).  The cell matrices are built once per chunk for all candidates; map_fn may be a
    thread pool's map over the chunk start indices."""
    nf, nc = mesh.ntrace, mesh.ncell
    cf, cs = mesh.cell_faces, mesh.cell_sign
    bnd = mesh.boundary
    cnt = np.bincount(cf.ravel(), minlength=nf)
    cands, outward = [], []
    for lam, u_b, pi in solutions:
        u_glob = np.bincount(cf.ravel(), weights=(cs * u_b).ravel(), minlength=nf) / cnt
        u_glob[bnd] = 0.0
        cands.append((lam, u_b, pi, u_glob))
        outward.append(np.bincount(cf.ravel(), weights=u_b.ravel(), minlength=nf))

    def work(s0):
        cells = np.arange(s0, min(nc, s0 + chunk))
        return chunk_contributions(cell_matrices, cf, cs, cells, r_ub_cells, r_pi_cells, cands)

    B = np.zeros(nf)
    acc = [dict(sl=np.zeros(nf), mu=np.zeros(nf), mu_abs=np.zeros(nf), mu_dev=np.zeros(nf), rp=np.zeros(nc),
                rp_abs=np.zeros(nc), rp_dev=np.zeros(nc)) for _ in cands]
    starts = list(range(0, nc, chunk))
    for s0, part in zip(starts, map_fn(work, starts)):
        f = part["faces"].ravel()
        B += np.bincount(f, weights=part["b"].ravel(), minlength=nf)
        for a, pc in zip(acc, part["cands"]):
            for key in ("sl", "mu", "mu_abs", "mu_dev"):
                a[key] += np.bincount(f, weights=pc[key].ravel(), minlength=nf)
            n = pc["rp"].shape[0]
            for key in ("rp", "rp_abs", "rp_dev"):
                a[key][s0 : s0 + n] = pc[key]
    bnorm = float(np.linalg.norm(B))
    rhs_u = np.bincount(cf.ravel(), weights=(cs * r_ub_cells).ravel(), minlength=nf)
    it = ~bnd
    res = []
    for a, ow in zip(acc, outward):
        berr_u = np.abs(rhs_u[it] - a["mu"][it]) / (a["mu_abs"][it] + np.abs(rhs_u[it]))
        berr_p = np.abs(a["rp"]) / a["rp_abs"]
        bound_u = a["mu_dev"][it] / (a["mu_abs"][it] + np.abs(rhs_u[it]))
        bound_p = a["rp_dev"] / a["rp_abs"]
        mres = np.sqrt(np.sum((rhs_u[it] - a["mu"][it]) ** 2) + np.sum(a["rp"] ** 2))
        rnorm = np.sqrt(np.sum(rhs_u[it] ** 2) + np.sum(r_pi_cells ** 2))
        res.append(dict(trace_res=float(np.linalg.norm(B - a["sl"])) / bnorm,
                        defect=float(np.abs(ow).max()) / bnorm, defect_norm=float(np.linalg.norm(ow)) / bnorm,
                        mixed_berr=max(float(berr_u.max()), float(berr_p.max())),
                        mixed_berr_bound=max(float(bound_u.max()), float(bound_p.max())), mixed_res=float(mres / rnorm),
                        bnorm=bnorm))
    return res


# ----- running the pass in its own process (a pool of forked workers over the chunks) -----

_JOB = {}


def _chunk_worker(s0):
    j = _JOB
    cells = np.arange(s0, min(j["mesh"].ncell, s0 + j["chunk"]))
    return chunk_contributions(j["cell_matrices"], j["mesh"].cell_faces, j["mesh"].cell_sign, cells, j["ruc"],
                               j["rpc"], j["cands"])


def _build(spec):
    """The synthetic problem, the oracle's mesh and its cell-matrix function for a spec dict."""
    from .local import local_matrices, shell_local_matrices
    from .mesh import BoxMesh, TableMesh

    if spec["kind"] == "sphere":
        from synth import make_sphere, make_rhs_sphere

        prob = make_sphere(spec["n"], spec["nlev"], dt=spec["dt"], mg_levels=spec["mg_levels"])
        mesh = TableMesh(prob.nlev, prob.col_edge, prob.edge_col, prob.edge_lf)
        return prob, mesh, (lambda cells: shell_local_matrices(mesh, prob, cells=cells)), make_rhs_sphere
    from synth import make_box, make_rhs

    prob = make_box(nx=spec["nx"], ny=spec["nx"], nlev=spec["nlev"], dx=spec["dx"], dz=spec["dz"], dt=spec["dt"],
                    mg_levels=spec["mg_levels"])
    mesh = BoxMesh(prob.nx, prob.ny, prob.nlev, prob.dx, prob.dy, prob.z)
    return prob, mesh, (lambda cells: local_matrices(mesh, prob, cells=cells)), make_rhs


def main(argv=None):
    """python -m oracle.allrows SPEC_JSON CANDIDATES_NPZ WORKERS: the residuals of the candidate
    solutions (arrays lam_i, ub_i (ncell, 6), pi_i) for the right-hand side of the given seed, as
    one JSON line."""
    import json
    import multiprocessing as mp
    import sys

    from .problem import cells_from_soa

    argv = sys.argv[1:] if argv is None else argv
    spec = json.loads(argv[0])
    data = np.load(argv[1])
    workers = int(argv[2])
    prob, mesh, cell_matrices, rhs = _build(spec)
    ruc, rpc = cells_from_soa(*rhs(prob, spec["seed"]))
    sols = [(data[f"lam{i}"], data[f"ub{i}"], data[f"pi{i}"]) for i in range(int(data["count"]))]
    nf = mesh.ntrace
    cf, cs = mesh.cell_faces, mesh.cell_sign
    cnt = np.bincount(cf.ravel(), minlength=nf)
    cands = []
    for lam, u_b, pi in sols:
        u_glob = np.bincount(cf.ravel(), weights=(cs * u_b).ravel(), minlength=nf) / cnt
        u_glob[mesh.boundary] = 0.0
        cands.append((lam, u_b, pi, u_glob))
    _JOB.update(mesh=mesh, cell_matrices=cell_matrices, ruc=ruc, rpc=rpc, cands=cands, chunk=32768)
    with mp.get_context("fork").Pool(workers) as pool:
        res = all_rows(cell_matrices, mesh, ruc, rpc, sols, chunk=32768,
                       map_fn=lambda f, starts: pool.imap(_chunk_worker, starts))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
