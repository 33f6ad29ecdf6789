"""Vertex-patch operators, dense-LU inverses and additive Schwarz (oracle).

A vertex patch is the 2x2x2 block of cells around an interior mesh vertex
(i, j, k), 1 <= i < n_x etc.  Its unknowns are the (2p-1)^3 global nodes
strictly inside the block, so the patch problem carries homogeneous Dirichlet
conditions on the block boundary.  Every cell containing such a node belongs
to the patch, so the patch operator is the assembled operator restricted to
those nodes:  A_P = R_P A_CG R_P^T, assembled here from the eight element
matrices by plain quadrature and factored by dense LU.

The additive Schwarz preconditioner is  P_AS r = sum_P R_P^T A_P^{-1} R_P r
acting on an assembled global residual r.  It consumes the residual only
through its assembly and returns a continuous field, the structure the paper's
Remark "Beyond DSS" (Section 3.2) requires of a consistent preconditioner.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .element import element_stiffness
from .mesh import Mesh


def interior_vertices(mesh: Mesh) -> np.ndarray:
    """All interior vertices (i, j, k), lexicographic with i fastest."""
    nx, ny, nz = mesh.n
    k, j, i = np.meshgrid(np.arange(1, nz), np.arange(1, ny), np.arange(1, nx), indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)


def patch_nodes(mesh: Mesh, v) -> np.ndarray:
    """Global nodes strictly inside the 2x2x2 block around vertex v, x fastest."""
    p = mesh.p
    i, j, k = (int(t) for t in v)
    nP = 2 * p - 1
    q = np.arange(nP)
    I = (i - 1) * p + 1 + q
    J = (j - 1) * p + 1 + q
    K = (k - 1) * p + 1 + q
    KK, JJ, II = np.meshgrid(K, J, I, indexing="ij")
    return mesh.gidx(II.ravel(), JJ.ravel(), KK.ravel())


def patch_matrix(mesh: Mesh, v) -> np.ndarray:
    """A_P assembled from the eight element matrices of the patch."""
    p = mesh.p
    n1 = p + 1
    nP = 2 * p - 1
    i, j, k = (int(t) for t in v)
    A = np.zeros((nP ** 3, nP ** 3))
    a = np.arange(n1 ** 3) % n1
    b = (np.arange(n1 ** 3) // n1) % n1
    c = np.arange(n1 ** 3) // (n1 * n1)
    for s3 in (0, 1):
        for s2 in (0, 1):
            for s1 in (0, 1):
                ci, cj, ck = i - 1 + s1, j - 1 + s2, k - 1 + s3
                Ae = element_stiffness(p, mesh.h[0][ci], mesh.h[1][cj], mesh.h[2][ck])
                # patch-local coordinate of each cell node (-1 = patch boundary)
                qx, qy, qz = a + s1 * p - 1, b + s2 * p - 1, c + s3 * p - 1
                ok = (qx >= 0) & (qx < nP) & (qy >= 0) & (qy < nP) & (qz >= 0) & (qz < nP)
                loc = np.where(ok, qx + nP * (qy + nP * qz), -1)
                idx = np.nonzero(ok)[0]
                A[np.ix_(loc[idx], loc[idx])] += Ae[np.ix_(idx, idx)]
    return A


def patch_solve(mesh: Mesh, v, r_local: np.ndarray) -> np.ndarray:
    """A_P^{-1} r_local by dense LU with partial pivoting."""
    lu = sla.lu_factor(patch_matrix(mesh, v))
    return sla.lu_solve(lu, r_local)


class SchwarzFactors:
    """Dense LU factors of every patch operator of a mesh, computed once."""

    def __init__(self, mesh: Mesh, vertices=None):
        self.mesh = mesh
        self.vertices = interior_vertices(mesh) if vertices is None else np.asarray(vertices)
        self.nodes = [patch_nodes(mesh, v) for v in self.vertices]
        self.lu = [sla.lu_factor(patch_matrix(mesh, v)) for v in self.vertices]

    def __call__(self, r: np.ndarray) -> np.ndarray:
        z = np.zeros(self.mesh.nglob)
        for idx, lu in zip(self.nodes, self.lu):
            z[idx] += sla.lu_solve(lu, r[idx])
        return z


def additive_schwarz(mesh: Mesh, r: np.ndarray, vertices=None) -> np.ndarray:
    """z = sum_P R_P^T A_P^{-1} R_P r on assembled global vectors."""
    if vertices is None:
        vertices = interior_vertices(mesh)
    z = np.zeros(mesh.nglob)
    for v in vertices:
        idx = patch_nodes(mesh, v)
        z[idx] += patch_solve(mesh, v, r[idx])
    return z


def additive_schwarz_at_cells(mesh: Mesh, r: np.ndarray, cells) -> np.ndarray:
    """P_AS r evaluated only at the nodes of the given cells ([len(cells), n1^3]).

    A node of cell (i, j, k) lies inside exactly those patches whose vertex is
    one of the cell's eight corners, so those (interior) corner patches give
    the complete value there.
    """
    cells = np.asarray(cells)
    ci, cj, ck = mesh.cell_ijk(cells)
    verts = set()
    for e in range(len(cells)):
        for dk in (0, 1):
            for dj in (0, 1):
                for di in (0, 1):
                    v = (ci[e] + di, cj[e] + dj, ck[e] + dk)
                    if (0 < v[0] < mesh.n[0]) and (0 < v[1] < mesh.n[1]) and (0 < v[2] < mesh.n[2]):
                        verts.add(v)
    z = np.zeros(mesh.nglob)
    for v in sorted(verts, key=lambda t: (t[2], t[1], t[0])):
        idx = patch_nodes(mesh, v)
        z[idx] += patch_solve(mesh, v, r[idx])
    return z[mesh.cell_dofs(cells)]
