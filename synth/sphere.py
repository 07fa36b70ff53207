"""Extruded equiangular cubed-sphere meshes, reference states and seeded right-hand sides.

Mesh conventions (the same interface as the periodic box of ``synth.box``):

* C_n mesh: six panels of n x n columns.  Column ``col = p n^2 + j n + i`` for
  panel p and panel coordinates (i, j); cells ``c = k * ncol + col``.
* Panel p has a right-handed frame (centre direction c_p, axes a_p, b_p with
  a_p x b_p = c_p, so the local frame of every column turns the same way
  seen from outside).  The point of panel coordinates (alpha, beta) in
  [-pi/4, pi/4]^2 is the direction of c_p + tan(alpha) a_p + tan(beta) b_p
  (equiangular grid: alpha and beta equally spaced).
* The local faces of a column follow its panel frame: W (alpha low), E, S
  (beta low), N; B and T as on the box.  Column corners are stored as unit
  vectors ``corners[q][d][col]`` for q = I + 2 J at panel offsets (I, J) in
  {0, 1}^2, d = x, y, z; cell corner (I, J, K) sits at radius[k + K] times
  corner q.
* Edges (the vertical faces seen from above): 2 ncol of them, numbered by the
  column the edge normal enters and its local face there; ``edge_col[0][e]``
  is the column the normal leaves.  The normal leaves through E or N when
  exactly one of the two local faces is E or N, else it leaves the column of
  lower index.
* Multigrid levels: C_n -> C_{n/2} by 2x2 agglomeration inside each panel; a
  coarse column keeps the panel frame of its children; children order (0,0),
  (1,0), (0,1), (1,1) in (i, j) offsets.

The reference state is the same synthetic stand-in as on the box, as a function
of the height above the ground z = r - radius_earth (horizontally uniform, so
that theta* is single valued on every facet).  The right-hand side adds a smooth
Gaussian bump of the pressure residual, centred at 45 E, 35 N with a 1000 km
width.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .box import CP, GRAV, RD, Level, reference_profiles

EARTH_RADIUS = 6371.0e3
OMEGA_EARTH = 7.292e-5

# (centre, alpha axis, beta axis) per panel, a x b = c
PANEL_FRAMES = np.array(
    [
        [[1, 0, 0], [0, 1, 0], [0, 0, 1]],
        [[0, 1, 0], [-1, 0, 0], [0, 0, 1]],
        [[-1, 0, 0], [0, -1, 0], [0, 0, 1]],
        [[0, -1, 0], [1, 0, 0], [0, 0, 1]],
        [[0, 0, 1], [0, 1, 0], [-1, 0, 0]],
        [[0, 0, -1], [0, 1, 0], [1, 0, 0]],
    ],
    np.float64,
)


@dataclass
class SphereLevel(Level):
    n: int = 0

    @property
    def ncol(self) -> int:
        return 6 * self.n * self.n

    @property
    def nedge(self) -> int:
        return 12 * self.n * self.n


def _tangents(n: int) -> np.ndarray:
    """tan of the n + 1 equiangular grid angles, exactly antisymmetric and exactly +-1 at the ends."""
    t = np.tan(np.pi / 4.0 * (2.0 * np.arange(n + 1) - n) / n)
    half = (n + 1) // 2
    t[n - np.arange(half)] = -t[np.arange(half)]
    t[0], t[n] = -1.0, 1.0
    if n % 2 == 0:
        t[n // 2] = 0.0
    return t


def cubed_sphere_tables(n: int):
    """Connectivity tables and corner unit vectors of the C_n mesh."""
    if n < 1:
        raise ValueError("C_n needs n >= 1")
    t = _tangents(n)
    ncol = 6 * n * n
    # vertex grid of every panel on the cube surface (exact at shared vertices)
    P = np.arange(6)[:, None, None]
    I = np.arange(n + 1)[None, None, :]
    J = np.arange(n + 1)[None, :, None]
    F = PANEL_FRAMES
    cube = (F[P, 0] + t[I][..., None] * F[P, 1] + t[J][..., None] * F[P, 2])  # (6, n+1 (j), n+1 (i), 3)
    flat = cube.reshape(-1, 3)
    _, vid = np.unique(flat, axis=0, return_inverse=True)
    vid = vid.reshape(6, n + 1, n + 1)
    unit = cube / np.linalg.norm(cube, axis=-1, keepdims=True)
    p = np.repeat(np.arange(6), n * n)
    jj = np.tile(np.repeat(np.arange(n), n), 6)
    ii = np.tile(np.arange(n), 6 * n)
    v = {(a, b): vid[p, jj + b, ii + a] for a in (0, 1) for b in (0, 1)}
    corners = np.empty((4, 3, ncol))
    for q, (a, b) in enumerate(((0, 0), (1, 0), (0, 1), (1, 1))):
        corners[q] = unit[p, jj + b, ii + a].T
    # the four faces W, E, S, N as vertex pairs
    faces = [(v[0, 0], v[0, 1]), (v[1, 0], v[1, 1]), (v[0, 0], v[1, 0]), (v[0, 1], v[1, 1])]
    keys = np.stack([np.minimum(a, b) * (flat.shape[0] + 1) + np.maximum(a, b) for a, b in faces])  # (4, ncol)
    ukeys, eid = np.unique(keys.ravel(), return_inverse=True)
    if ukeys.shape[0] != 2 * ncol:
        raise RuntimeError("cubed sphere: wrong number of edges")
    eid = eid.reshape(4, ncol)
    cols = np.tile(np.arange(ncol), 4)
    lfs = np.repeat(np.arange(4), ncol)
    order = np.argsort(eid.ravel(), kind="stable")
    e_sorted = eid.ravel()[order]
    if not np.all(e_sorted[0::2] == e_sorted[1::2]) or not np.all(np.diff(e_sorted[0::2]) == 1):
        raise RuntimeError("cubed sphere: every edge needs exactly two columns")
    ca, cb = cols[order][0::2], cols[order][1::2]
    la, lb = lfs[order][0::2], lfs[order][1::2]
    odd_a, odd_b = la % 2 == 1, lb % 2 == 1
    a_leaves = np.where(odd_a != odd_b, odd_a, ca < cb)
    c0, c1 = np.where(a_leaves, ca, cb), np.where(a_leaves, cb, ca)
    l0, l1 = np.where(a_leaves, la, lb), np.where(a_leaves, lb, la)
    # number the edges by the column the normal enters, then its local face there
    perm = np.lexsort((l1, c1))
    c0, c1, l0, l1 = c0[perm], c1[perm], l0[perm], l1[perm]
    edge_col = np.stack([c0, c1]).astype(np.int32)
    edge_lf = np.stack([l0, l1]).astype(np.int32)
    col_edge = np.empty((4, ncol), np.int32)
    e = np.arange(2 * ncol)
    col_edge[l0, c0] = e
    col_edge[l1, c1] = e
    return col_edge, edge_col, edge_lf, corners


def sphere_hierarchy(n: int, nlevels: int) -> list:
    levels = []
    ce, ec, el, _ = cubed_sphere_tables(n)
    levels.append(SphereLevel(0, 0, ce, ec, el, n=n))
    for _ in range(1, nlevels):
        fn = levels[-1].n
        if fn % 2:
            raise ValueError(f"cannot coarsen C{fn} by 2x2")
        cn = fn // 2
        ce, ec, el, _ = cubed_sphere_tables(cn)
        fcol = np.arange(6 * fn * fn)
        p, r = fcol // (fn * fn), fcol % (fn * fn)
        j, i = r // fn, r % fn
        parent = p * cn * cn + (j // 2) * cn + i // 2
        ccol = np.arange(6 * cn * cn)
        cp_, cr = ccol // (cn * cn), ccol % (cn * cn)
        J, I = cr // cn, cr % cn
        children = np.stack([cp_ * fn * fn + (2 * J + dj) * fn + 2 * I + di
                             for (di, dj) in ((0, 0), (1, 0), (0, 1), (1, 1))])
        levels.append(SphereLevel(0, 0, ce, ec, el, parent.astype(np.int32), children.astype(np.int32), n=cn))
    return levels


@dataclass
class SphereProblem:
    n: int
    nlev: int
    z: np.ndarray  # [nlev+1] interface heights above the ground
    radius: np.ndarray  # [nlev+1] interface radii
    corners: np.ndarray  # [4][3][ncol] unit vectors
    levels: list
    theta_w: np.ndarray
    exner_hat_w: np.ndarray
    exner_c: np.ndarray
    rho_c: np.ndarray
    dt: float
    omega_rot: float = OMEGA_EARTH
    tau_u: float = 0.5
    tau_rho: float = 0.5
    tau_theta: float = 0.5
    cp: float = CP
    rd: float = RD
    grav: float = GRAV
    meta: dict = field(default_factory=dict)
    geom: str = "shell"
    dx: float = 0.0
    dy: float = 0.0

    @property
    def ncol(self) -> int:
        return 6 * self.n * self.n

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

    def column_centres(self) -> np.ndarray:
        """Unit vectors (3, ncol) towards the column centres (normalised mean of the corners)."""
        m = self.corners.mean(axis=0)
        return m / np.linalg.norm(m, axis=0, keepdims=True)


def make_sphere(
    n: int,
    nlev: int,
    *,
    ztop: float = 30.0e3,
    stretch: str = "quadratic",
    dt: float = 1800.0,
    radius_earth: float = EARTH_RADIUS,
    omega_rot: float = OMEGA_EARTH,
    cs: float = 340.0,
    nbv: float = 0.01,
    rho_scale_height: float = 8000.0,
    rho0: float = 1.2,
    mg_levels: int = 4,
    perturb: float = 0.0,
    seed: int = 0,
    tau: float = 0.5,
) -> SphereProblem:
    """Extruded C_n cubed sphere with layers to ``ztop`` (z_k = ztop (k/L)^2, or uniform)."""
    if stretch == "quadratic":
        z = ztop * (np.arange(nlev + 1, dtype=np.float64) / nlev) ** 2
    elif stretch == "uniform":
        z = ztop * np.arange(nlev + 1, dtype=np.float64) / nlev
    else:
        raise ValueError(stretch)
    levels = sphere_hierarchy(n, mg_levels)
    _, _, _, corners = cubed_sphere_tables(n)
    ncol = 6 * n * n
    theta_1d, exner_1d, t0 = reference_profiles(z, cs=cs, nbv=nbv)
    zc = 0.5 * (z[1:] + z[:-1])
    theta_c1d, _, _ = reference_profiles(zc, cs=cs, nbv=nbv)
    theta_w = np.repeat(theta_1d[:, None], ncol, axis=1)
    exner_hat_w = np.repeat(exner_1d[:, None], ncol, axis=1)
    exner_c = np.repeat((t0 / theta_c1d)[:, None], ncol, axis=1)
    rho_c = np.repeat((rho0 * np.exp(-zc / rho_scale_height))[:, None], ncol, axis=1)
    if perturb:
        rng = np.random.default_rng(seed + 7919)
        exner_c = exner_c * (1.0 + perturb * rng.uniform(-1.0, 1.0, exner_c.shape))
    return SphereProblem(
        n=n,
        nlev=nlev,
        z=z,
        radius=radius_earth + z,
        corners=np.ascontiguousarray(corners),
        levels=levels,
        theta_w=np.ascontiguousarray(theta_w),
        exner_hat_w=np.ascontiguousarray(exner_hat_w),
        exner_c=np.ascontiguousarray(exner_c),
        rho_c=np.ascontiguousarray(rho_c),
        dt=float(dt),
        omega_rot=float(omega_rot),
        tau_u=tau,
        tau_rho=tau,
        tau_theta=tau,
        meta=dict(cs=cs, nbv=nbv, t0=t0, seed=seed, theta_single_valued=True, radius_earth=radius_earth),
    )


def make_rhs_sphere(prob: SphereProblem, seed: int, bump: float = 10.0, bump_width: float = 1000.0e3,
                    bump_lon_deg: float = 45.0, bump_lat_deg: float = 35.0):
    """Broken velocity residual [6][L][ncol] and pressure residual [L][ncol]: standard normal
    draws in the order (L, ncol, 6) then (L, ncol), plus bump * exp(-d^2 / (2 w^2)) on the
    pressure residual of every layer, d the great-circle distance at the ground from the bump
    centre to the column centre."""
    rng = np.random.default_rng(seed)
    ru = rng.standard_normal((prob.nlev, prob.ncol, 6))
    rp = rng.standard_normal((prob.nlev, prob.ncol))
    if bump:
        lon, lat = np.radians(bump_lon_deg), np.radians(bump_lat_deg)
        c0 = np.array([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)])
        cc = prob.column_centres()
        ang = np.arccos(np.clip(c0 @ cc, -1.0, 1.0))
        d = prob.meta.get("radius_earth", EARTH_RADIUS) * ang
        rp = rp + bump * np.exp(-d * d / (2.0 * bump_width * bump_width))[None, :]
    return np.ascontiguousarray(ru.transpose(2, 0, 1)), np.ascontiguousarray(rp)


def config_sphere(name: str, **kw) -> SphereProblem:
    """Named workloads: ``c192`` (C192 x 30 quadratic layers to 30 km, dt = 1800 s) and ``c384``
    (C384 x 70 quadratic layers to 30 km, dt = 900 s); radius 6371 km, Omega = 7.292e-5 /s."""
    if name == "c192":
        args = dict(n=192, nlev=30, dt=1800.0)
    elif name == "c384":
        args = dict(n=384, nlev=70, dt=900.0)
    else:
        raise KeyError(name)
    args.update(kw)
    return make_sphere(**args)
