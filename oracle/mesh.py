"""The oracle's own dof maps for a periodic extruded box (test infrastructure).

Numbering convention (the documented layout of trace vectors, shared as a
convention with the library's header, not as code):

* cells: ``k * ncol + iy * nx + ix``
* trace faces: first the horizontal facets (bottom/top of cells),
  ``k * ncol + col`` for k = 0..L, then the vertical facets,
  ``(L + 1) * ncol + k * 2 ncol + e`` with x-facet ``e = iy*nx + ix`` on the
  west side of column (ix, iy) and y-facet ``e = ncol + iy*nx + ix`` on its
  south side.
* local faces of a cell: W, E, S, N, B, T.
* global orientation of a facet normal: +x, +y, +z.
"""

from __future__ import annotations

import numpy as np


class BoxMesh:
    def __init__(self, nx, ny, nlev, dx, dy, z):
        self.nx, self.ny, self.nlev = int(nx), int(ny), int(nlev)
        self.dx, self.dy = float(dx), float(dy)
        self.z = np.asarray(z, np.float64)
        self.dz = np.diff(self.z)
        self.ncol = self.nx * self.ny
        self.ncell = self.ncol * self.nlev
        self.n_zface = self.ncol * (self.nlev + 1)
        self.n_hface = 2 * self.ncol * self.nlev
        self.ntrace = self.n_zface + self.n_hface
        self._build()

    def zface(self, k, ix, iy):
        return k * self.ncol + (iy % self.ny) * self.nx + (ix % self.nx)

    def xface(self, k, ix, iy):
        return self.n_zface + k * 2 * self.ncol + (iy % self.ny) * self.nx + (ix % self.nx)

    def yface(self, k, ix, iy):
        return self.n_zface + k * 2 * self.ncol + self.ncol + (iy % self.ny) * self.nx + (ix % self.nx)

    def _build(self):
        L, nx, ny, ncol = self.nlev, self.nx, self.ny, self.ncol
        c = np.arange(self.ncell)
        k = c // ncol
        col = c % ncol
        ix, iy = col % nx, col // nx
        faces = np.stack(
            [
                self.xface(k, ix, iy),
                self.xface(k, ix + 1, iy),
                self.yface(k, ix, iy),
                self.yface(k, ix, iy + 1),
                self.zface(k, ix, iy),
                self.zface(k + 1, ix, iy),
            ],
            axis=1,
        ).astype(np.int64)
        # the +x/+y/+z normal leaves the cell through E, N, T
        sign = np.tile(np.array([-1.0, 1.0, -1.0, 1.0, -1.0, 1.0]), (self.ncell, 1))
        self.cell_faces = faces
        self.cell_sign = sign
        self.cell_layer = k
        self.cell_ix = ix
        self.cell_iy = iy
        # a facet is on the rigid lid / ground when it is the bottom of layer 0 or the top of layer L-1
        bnd = np.zeros(self.ntrace, bool)
        bnd[:ncol] = True
        bnd[L * ncol : (L + 1) * ncol] = True
        self.boundary = bnd

    def face_cells(self):
        """For every trace facet the (cell, local face) pairs touching it: arrays (ntrace, 2), -1 if absent."""
        flat = self.cell_faces.ravel()
        order = np.argsort(flat, kind="stable")
        fsorted = flat[order]
        cells = np.full((self.ntrace, 2), -1, np.int64)
        lfs = np.full((self.ntrace, 2), -1, np.int64)
        first = np.ones(flat.shape[0], bool)
        first[1:] = fsorted[1:] != fsorted[:-1]
        slot = np.where(first, 0, 1)
        cells[fsorted, slot] = order // 6
        lfs[fsorted, slot] = order % 6
        return cells, lfs

    def column_of_zface(self, f):
        return f % self.ncol

    def is_zface(self, f):
        return f < self.n_zface


class TableMesh:
    """The dof maps of an extruded mesh given by its horizontal connectivity tables (the cubed
    sphere; the periodic box gives the same maps as ``BoxMesh``).

    Same numbering as the box: cells ``k * ncol + col``; horizontal facets ``k * ncol + col``;
    vertical facets ``(L + 1) * ncol + k * nedge + e``; local faces W, E, S, N, B, T in the
    column's own frame.  The global normal of edge e leaves ``edge_col[0][e]``; +z on B / T.
    ``parents`` (optional): for each multigrid level below the finest, the coarse column of every
    column of the level above it.
    """

    def __init__(self, nlev, col_edge, edge_col, edge_lf, parents=()):
        self.nlev = int(nlev)
        self.col_edge = np.asarray(col_edge, np.int64)
        self.edge_col = np.asarray(edge_col, np.int64)
        self.edge_lf = np.asarray(edge_lf, np.int64)
        self.ncol = self.col_edge.shape[1]
        self.nedge = self.edge_col.shape[1]
        self.ncell = self.ncol * self.nlev
        self.n_zface = self.ncol * (self.nlev + 1)
        self.n_hface = self.nedge * self.nlev
        self.ntrace = self.n_zface + self.n_hface
        self.parents = [np.asarray(p, np.int64) for p in parents]
        L, ncol = self.nlev, self.ncol
        c = np.arange(self.ncell)
        k, col = c // ncol, c % ncol
        faces = np.empty((self.ncell, 6), np.int64)
        sign = np.empty((self.ncell, 6))
        for f in range(4):
            e = self.col_edge[f, col]
            faces[:, f] = self.n_zface + k * self.nedge + e
            leaves = (self.edge_col[0, e] == col) & (self.edge_lf[0, e] == f)
            sign[:, f] = np.where(leaves, 1.0, -1.0)
        faces[:, 4] = k * ncol + col
        faces[:, 5] = (k + 1) * ncol + col
        sign[:, 4], sign[:, 5] = -1.0, 1.0
        self.cell_faces = faces
        self.cell_sign = sign
        self.cell_layer = k
        self.cell_col = col
        bnd = np.zeros(self.ntrace, bool)
        bnd[:ncol] = True
        bnd[L * ncol : (L + 1) * ncol] = True
        self.boundary = bnd

    face_cells = BoxMesh.face_cells

    def column_of_zface(self, f):
        return f % self.ncol

    def is_zface(self, f):
        return f < self.n_zface
