"""Periodic extruded box meshes, reference states and seeded right-hand sides.

Mesh conventions (the interface both sides of the solver agree on):

* Columns ``col = iy * nx + ix``; cells ``c = k * ncol + col`` (layer k = 0 is
  at the ground).  Every per-cell array is stored ``[k][col]``.
* Each column has four vertical faces ("edges" of the horizontal mesh) in the
  local order W, E, S, N (local face 0..3); the bottom and top faces of a cell
  are local faces 4 (B) and 5 (T).
* Horizontal-mesh edges: ``e in [0, ncol)`` are x-edges, edge ``iy*nx+ix`` lies
  on the west side of column (ix, iy); ``e in [ncol, 2 ncol)`` are y-edges,
  edge ``ncol + iy*nx+ix`` lies on the south side of column (ix, iy).  The
  mesh is periodic in x and y.
* ``edge_col[0][e]`` is the column the edge normal leaves (west / south),
  ``edge_col[1][e]`` the column it enters; ``edge_lf[s][e]`` is the local face
  index (0..3) of edge e inside ``edge_col[s][e]``.
* ``col_edge[f][col]`` is the edge of local face f (0..3) of a column.

Multigrid hierarchy: level l+1 agglomerates 2x2 columns of level l, with no
vertical coarsening.  ``parent[col_fine]`` gives the coarse column and
``children[q][col_coarse]`` (q = 0..3, order (0,0), (1,0), (0,1), (1,1) in
(ix, iy) offsets) the four fine columns.  A coarse column keeps the local face
orientation of its children.

Reference state (a synthetic stand-in for the model state, which is not part
of the method): potential temperature with constant buoyancy frequency N,
hydrostatic Exner pressure for that profile on the same vertically continuous
points, a cell Exner pressure giving a fixed temperature T0 = c_s^2 (1-kappa)/R
(sound speed c_s), and an exponentially decaying density.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CP = 1005.0
RD = 287.05
GRAV = 9.80665


@dataclass
class Level:
    nx: int
    ny: int
    col_edge: np.ndarray  # int32 [4, ncol]
    edge_col: np.ndarray  # int32 [2, nedge]
    edge_lf: np.ndarray  # int32 [2, nedge]
    parent: np.ndarray | None = None  # int32 [ncol_finer] (None on level 0)
    children: np.ndarray | None = None  # int32 [4, ncol] (None on level 0)

    @property
    def ncol(self) -> int:
        return self.nx * self.ny

    @property
    def nedge(self) -> int:
        return 2 * self.nx * self.ny


@dataclass
class BoxProblem:
    nx: int
    ny: int
    nlev: int
    dx: float
    dy: float
    z: np.ndarray  # [nlev+1] interface heights
    levels: list  # list[Level], levels[0] is the fine mesh
    theta_w: np.ndarray  # [nlev+1, ncol] potential temperature at bottom/top face points
    exner_hat_w: np.ndarray  # [nlev+1, ncol] Exner pressure projected to the same points
    exner_c: np.ndarray  # [nlev, ncol] cell Exner pressure
    rho_c: np.ndarray  # [nlev, ncol] cell density
    dt: float
    tau_u: float = 0.5
    tau_rho: float = 0.5
    tau_theta: float = 0.5
    cp: float = CP
    rd: float = RD
    grav: float = GRAV
    meta: dict = field(default_factory=dict)

    @property
    def ncol(self) -> int:
        return self.nx * self.ny

    @property
    def nedge(self) -> int:
        return 2 * self.ncol

    @property
    def ncell(self) -> int:
        return self.nlev * self.ncol

    @property
    def ntrace(self) -> int:
        return (self.nlev + 1) * self.ncol + self.nlev * self.nedge

    @property
    def kappa(self) -> float:
        return self.rd / self.cp

    @property
    def dz(self) -> np.ndarray:
        return np.diff(self.z)

    @property
    def col_edge(self):
        return self.levels[0].col_edge

    @property
    def edge_col(self):
        return self.levels[0].edge_col

    @property
    def edge_lf(self):
        return self.levels[0].edge_lf


def box_tables(nx: int, ny: int):
    """Connectivity tables of a periodic nx x ny quadrilateral mesh."""
    if nx < 2 or ny < 2:
        raise ValueError("periodic box needs nx, ny >= 2")
    ncol = nx * ny
    ix = np.arange(ncol) % nx
    iy = np.arange(ncol) // nx
    col = lambda i, j: (j % ny) * nx + (i % nx)  # noqa: E731
    col_edge = np.empty((4, ncol), np.int32)
    col_edge[0] = iy * nx + ix  # W: x-edge of this column
    col_edge[1] = col(ix + 1, iy)  # E: x-edge of the east neighbour
    col_edge[2] = ncol + iy * nx + ix  # S
    col_edge[3] = ncol + col(ix, iy + 1)  # N
    nedge = 2 * ncol
    edge_col = np.empty((2, nedge), np.int32)
    edge_lf = np.empty((2, nedge), np.int32)
    # x-edges: minus side = west column (edge is its E face), plus = east column (W face)
    edge_col[0, :ncol] = col(ix - 1, iy)
    edge_col[1, :ncol] = np.arange(ncol)
    edge_lf[0, :ncol] = 1
    edge_lf[1, :ncol] = 0
    # y-edges: minus = south column (N face), plus = north column (S face)
    edge_col[0, ncol:] = col(ix, iy - 1)
    edge_col[1, ncol:] = np.arange(ncol)
    edge_lf[0, ncol:] = 3
    edge_lf[1, ncol:] = 2
    return col_edge, edge_col, edge_lf


def box_hierarchy(nx: int, ny: int, nlevels: int) -> list:
    levels = []
    ce, ec, el = box_tables(nx, ny)
    levels.append(Level(nx, ny, ce, ec, el))
    for _ in range(1, nlevels):
        fx, fy = levels[-1].nx, levels[-1].ny
        if fx % 2 or fy % 2 or fx // 2 < 2 or fy // 2 < 2:
            raise ValueError(f"cannot coarsen a {fx}x{fy} level by 2x2")
        cx, cy = fx // 2, fy // 2
        ce, ec, el = box_tables(cx, cy)
        fcol = np.arange(fx * fy)
        parent = ((fcol // fx) // 2) * cx + (fcol % fx) // 2
        ccol = np.arange(cx * cy)
        I, J = ccol % cx, ccol // cx
        children = np.stack([(2 * J + dj) * fx + 2 * I + di for (di, dj) in ((0, 0), (1, 0), (0, 1), (1, 1))])
        levels.append(Level(cx, cy, ce, ec, el, parent.astype(np.int32), children.astype(np.int32)))
    return levels


def reference_profiles(z, *, cs, nbv, theta_s=None, rd=RD, cp=CP, grav=GRAV):
    """theta(z) with constant buoyancy frequency and the hydrostatic Exner pressure."""
    kappa = rd / cp
    t0 = cs * cs * (1.0 - kappa) / rd
    if theta_s is None:
        theta_s = t0
    z = np.asarray(z, np.float64)
    if nbv == 0.0:
        theta = np.full_like(z, theta_s)
        exner = 1.0 - grav * z / (cp * theta_s)
    else:
        n2 = nbv * nbv
        theta = theta_s * np.exp(n2 * z / grav)
        exner = 1.0 - grav * grav / (cp * theta_s * n2) * (1.0 - np.exp(-n2 * z / grav))
    return theta, exner, t0


def make_box(
    nx: int,
    ny: int,
    nlev: int,
    dx: float,
    dy: float | None = None,
    dz: float | None = None,
    *,
    ztop: float | None = None,
    stretch: str = "uniform",
    dt: float = 600.0,
    cs: float = 340.0,
    nbv: float = 0.01,
    rho_scale_height: float = 8000.0,
    rho0: float = 1.2,
    mg_levels: int = 4,
    perturb: float = 0.0,
    theta_col_perturb: float = 0.0,
    seed: int = 0,
    tau: float = 0.5,
) -> BoxProblem:
    """Build a periodic extruded box problem.

    ``perturb`` multiplies the cell Exner pressure by ``1 + perturb * U(-1,1)``
    per cell (seeded), which makes the pressure mass term vary from cell to
    cell.  ``theta_col_perturb`` scales theta per column; it breaks the
    single-valuedness of theta on vertical faces, so it is only for tests of
    the hybridised operator on its own.
    """
    if dy is None:
        dy = dx
    if stretch == "uniform":
        if dz is None:
            raise ValueError("uniform layers need dz")
        z = dz * np.arange(nlev + 1, dtype=np.float64)
    elif stretch == "quadratic":
        if ztop is None:
            raise ValueError("quadratic stretching needs ztop")
        z = ztop * (np.arange(nlev + 1, dtype=np.float64) / nlev) ** 2
    else:
        raise ValueError(stretch)
    levels = box_hierarchy(nx, ny, mg_levels)
    ncol = nx * ny
    theta_1d, exner_1d, t0 = reference_profiles(z, cs=cs, nbv=nbv)
    zc = 0.5 * (z[1:] + z[:-1])
    theta_c1d, _, _ = reference_profiles(zc, cs=cs, nbv=nbv)
    theta_w = np.repeat(theta_1d[:, None], ncol, axis=1)
    exner_hat_w = np.repeat(exner_1d[:, None], ncol, axis=1)
    exner_c = np.repeat((t0 / theta_c1d)[:, None], ncol, axis=1)
    rho_c = np.repeat((rho0 * np.exp(-zc / rho_scale_height))[:, None], ncol, axis=1)
    rng = np.random.default_rng(seed + 7919)
    if perturb:
        exner_c = exner_c * (1.0 + perturb * rng.uniform(-1.0, 1.0, exner_c.shape))
    if theta_col_perturb:
        theta_w = theta_w * (1.0 + theta_col_perturb * rng.uniform(-1.0, 1.0, (1, ncol)))
    return BoxProblem(
        nx=nx,
        ny=ny,
        nlev=nlev,
        dx=float(dx),
        dy=float(dy),
        z=z,
        levels=levels,
        theta_w=np.ascontiguousarray(theta_w),
        exner_hat_w=np.ascontiguousarray(exner_hat_w),
        exner_c=np.ascontiguousarray(exner_c),
        rho_c=np.ascontiguousarray(rho_c),
        dt=float(dt),
        tau_u=tau,
        tau_rho=tau,
        tau_theta=tau,
        meta=dict(cs=cs, nbv=nbv, t0=t0, seed=seed, theta_single_valued=theta_col_perturb == 0.0),
    )


def make_rhs(prob: BoxProblem, seed: int):
    """Dual right-hand side: broken velocity part [6][L][ncol] and pressure part [L][ncol].

    Draw order: the broken velocity residual of shape (L, ncol, 6), then the
    pressure residual of shape (L, ncol), both standard normal, C order.
    """
    rng = np.random.default_rng(seed)
    ru = rng.standard_normal((prob.nlev, prob.ncol, 6))
    rp = rng.standard_normal((prob.nlev, prob.ncol))
    return np.ascontiguousarray(ru.transpose(2, 0, 1)), np.ascontiguousarray(rp)


def make_rhs_p1(prob: BoxProblem, seed: int):
    """Dual right-hand side of the order-1 system: broken RT1 velocity part [36][L][ncol] and DG1
    pressure part [8][L][ncol].  Draw order: (L, ncol, 36) then (L, ncol, 8), standard normal."""
    rng = np.random.default_rng(seed)
    ru = rng.standard_normal((prob.nlev, prob.ncol, 36))
    rp = rng.standard_normal((prob.nlev, prob.ncol, 8))
    return np.ascontiguousarray(ru.transpose(2, 0, 1)), np.ascontiguousarray(rp.transpose(2, 0, 1))


def config_box(name: str, **kw) -> BoxProblem:
    """Named workloads.

    * ``box16``: periodic 16x16x8, dx = 10 km, dz = 1.25 km, dt = 600 s.
    * ``box256``: periodic 256x256x64, dx = 5 km, dz = 250 m, dt = 600 s.
    Both: isothermal-sound-speed state c_s = 340 m/s, N = 0.01 /s,
    density scale height 8 km, 4 multigrid levels.
    """
    if name == "box16":
        args = dict(nx=16, ny=16, nlev=8, dx=10e3, dz=1250.0)
    elif name == "box256":
        args = dict(nx=256, ny=256, nlev=64, dx=5e3, dz=250.0)
    else:
        raise KeyError(name)
    args.update(kw)
    return make_box(**args)
