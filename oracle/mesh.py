"""Graded Cartesian hexahedral mesh and its global/cell-wise numbering (oracle).

Global nodes are numbered lexicographically with x fastest,
``g = I + Nx * (J + Ny * K)`` with ``Nd = n_d * p + 1``.  Cells are numbered
``e = i + n_x * (j + n_y * k)``; the local node (a, b, c) of a cell (a along
x) has local index ``a + (p+1) * (b + (p+1) * c)`` and global node
``(i p + a, j p + b, k p + c)``.  The array ``dofs[e, l]`` is the gather
operator G of Section 2.1 written as an index map.
"""
from __future__ import annotations

import numpy as np

from .basis import gll_nodes


class Mesh:
    def __init__(self, p: int, n, widths=None):
        if isinstance(n, (int, np.integer)):
            n = (int(n),) * 3
        self.p = int(p)
        self.n = tuple(int(v) for v in n)
        if widths is None:
            widths = [np.full(nd, 1.0 / nd) for nd in self.n]
        self.h = [np.asarray(w, dtype=float).copy() for w in widths]
        for d in range(3):
            assert self.h[d].shape == (self.n[d],) and np.all(self.h[d] > 0)
        self.n1 = self.p + 1
        self.N = tuple(nd * self.p + 1 for nd in self.n)
        self.nglob = self.N[0] * self.N[1] * self.N[2]
        self.ncells = self.n[0] * self.n[1] * self.n[2]
        self.vertices = [np.concatenate(([0.0], np.cumsum(hd))) for hd in self.h]
        self._dofs = None

    # ---- numbering -------------------------------------------------------
    def gidx(self, I, J, K):
        return I + self.N[0] * (J + self.N[1] * K)

    def cell_ijk(self, e):
        e = np.asarray(e)
        i = e % self.n[0]
        j = (e // self.n[0]) % self.n[1]
        k = e // (self.n[0] * self.n[1])
        return i, j, k

    def local_abc(self):
        n1 = self.n1
        l = np.arange(n1 ** 3)
        return l % n1, (l // n1) % n1, l // (n1 * n1)

    @property
    def dofs(self) -> np.ndarray:
        """dofs[e, l]: global node of local node l of cell e."""
        if self._dofs is None:
            i, j, k = self.cell_ijk(np.arange(self.ncells))
            a, b, c = self.local_abc()
            p = self.p
            self._dofs = self.gidx(i[:, None] * p + a[None, :],
                                   j[:, None] * p + b[None, :],
                                   k[:, None] * p + c[None, :])
        return self._dofs

    def cell_dofs(self, cells) -> np.ndarray:
        cells = np.asarray(cells)
        i, j, k = self.cell_ijk(cells)
        a, b, c = self.local_abc()
        p = self.p
        return self.gidx(i[:, None] * p + a[None, :], j[:, None] * p + b[None, :],
                         k[:, None] * p + c[None, :])

    # ---- geometry --------------------------------------------------------
    def coords_1d(self, d: int) -> np.ndarray:
        """Coordinates of the N_d global node planes along direction d."""
        xi = gll_nodes(self.p)
        X = np.empty(self.N[d])
        for i in range(self.n[d]):
            X[i * self.p:(i + 1) * self.p + 1] = self.vertices[d][i] + self.h[d][i] * xi
        # make shared vertex planes exactly the cumulative vertex coordinate
        X[::self.p] = self.vertices[d]
        return X

    def cell_sizes(self, cells=None):
        if cells is None:
            cells = np.arange(self.ncells)
        i, j, k = self.cell_ijk(cells)
        return self.h[0][i], self.h[1][j], self.h[2][k]

    def boundary_mask(self) -> np.ndarray:
        """True at global nodes on the boundary of the box."""
        I = np.arange(self.nglob) % self.N[0]
        J = (np.arange(self.nglob) // self.N[0]) % self.N[1]
        K = np.arange(self.nglob) // (self.N[0] * self.N[1])
        return ((I == 0) | (I == self.N[0] - 1) | (J == 0) | (J == self.N[1] - 1)
                | (K == 0) | (K == self.N[2] - 1))

    def multiplicity(self) -> np.ndarray:
        """Number of cells sharing each global node."""
        return np.bincount(self.dofs.ravel(), minlength=self.nglob)
