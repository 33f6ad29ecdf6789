"""Two-level preconditioner: the vertex-patch Schwarz smoother on Q_p plus an
exact coarse correction on the Q_1 space of the same mesh (oracle; test
infrastructure).

The paper names a multigrid V-cycle that consumes its input only through the
assembled residual G^T r as the preconditioner its solver is built for
(Remark after the Theorem "Equivalence of Communication-Free FCG", and the
Conclusions); the multigrid itself is in a companion paper that is not
available.  This is the textbook two-level member of that family, written
from its definition on assembled global vectors:

* coarse space V_0 = continuous piecewise trilinear functions on the same
  hexahedral mesh, zero on the Dirichlet boundary.  V_0 is a subspace of
  the Q_p space, so its prolongation P_0 is plain interpolation: column v
  of P_0 holds the values of the trilinear hat function of interior vertex v
  at the Q_p nodes (a product of 1D hats evaluated at the node coordinates);
* coarse operator A_0 = P_0^T A_D P_0 (Galerkin), solved exactly (sparse LU);
* one application, from z = 0: `pre` damped Richardson sweeps on additive
  Schwarz, the coarse correction z <- z + P_0 A_0^{-1} P_0^T (r - A z), then
  `post` sweeps, z <- z + omega P_AS (r - A z).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import Mesh
from .operators import apply_global, assemble
from .patches import SchwarzFactors


def hat_values(vertices: np.ndarray, x: np.ndarray) -> np.ndarray:
    """[len(x), len(vertices)]: the 1D piecewise-linear hat function of each
    vertex evaluated at the points x (which lie inside the vertex range)."""
    H = np.zeros((len(x), len(vertices)))
    for v in range(len(vertices)):
        if v > 0:
            a, b = vertices[v - 1], vertices[v]
            m = (x >= a) & (x <= b)
            H[m, v] = (x[m] - a) / (b - a)
        if v < len(vertices) - 1:
            a, b = vertices[v], vertices[v + 1]
            m = (x >= a) & (x <= b)
            H[m, v] = np.maximum(H[m, v], (b - x[m]) / (b - a))
    return H


def coarse_vertices(mesh: Mesh):
    """Interior vertices (i, j, k), 1 <= i < n_x etc., lexicographic i fastest."""
    nx, ny, nz = mesh.n
    k, j, i = np.meshgrid(np.arange(1, nz), np.arange(1, ny), np.arange(1, nx), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def prolongation(mesh: Mesh) -> sp.csr_matrix:
    """P_0: coarse interior-vertex values -> Q_p nodal values (nglob x nv)."""
    H = [hat_values(mesh.vertices[d], mesh.coords_1d(d)) for d in range(3)]
    # interior vertices only (Dirichlet)
    H = [sp.csr_matrix(h[:, 1:-1]) for h in H]
    # global node g = I + N0 (J + N1 K), vertex v = i + m0 (j + m1 k): Kronecker
    # order with x fastest
    return sp.kron(sp.kron(H[2], H[1]), H[0]).tocsr()


class TwoLevel:
    """The two-level preconditioner of a mesh, factors computed once."""

    def __init__(self, mesh: Mesh, omega: float = 0.125, pre: int = 1, post: int = 1):
        self.mesh = mesh
        self.omega, self.pre, self.post = omega, pre, post
        self.P0 = prolongation(mesh)
        A = assemble(mesh, dirichlet=True)
        self.A0 = (self.P0.T @ A @ self.P0).tocsc()
        self.lu = spla.splu(self.A0) if self.A0.shape[0] > 0 else None
        self.schwarz = SchwarzFactors(mesh)

    def coarse(self, r: np.ndarray) -> np.ndarray:
        """P_0 A_0^{-1} P_0^T r."""
        if self.lu is None:
            return np.zeros_like(r)
        return self.P0 @ self.lu.solve(self.P0.T @ r)

    def __call__(self, r: np.ndarray) -> np.ndarray:
        m = self.mesh
        z = np.zeros_like(r)
        for _ in range(self.pre):
            z = z + self.omega * self.schwarz(r - apply_global(m, z))
        z = z + self.coarse(r - apply_global(m, z))
        for _ in range(self.post):
            z = z + self.omega * self.schwarz(r - apply_global(m, z))
        return z
