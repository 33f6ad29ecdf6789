"""Gather/scatter, DSS and the Dirichlet Laplacian apply (oracle).

* ``gather``  -- G: global primal vector -> cell-wise copies (Section 2.1).
* ``scatter`` -- G^T: cell-wise dual contributions -> assembled global vector.
* ``dss``     -- S = G G^T (Section 3.3): every copy receives the sum of all
  copies of its node.
* ``apply_global`` -- y = A_D x with A_D = P_I A_CG P_I: the assembled Laplacian
  with homogeneous Dirichlet conditions imposed by masking (boundary rows and
  columns zero).  With ``dirichlet=False`` it is the plain (Neumann) A_CG.
* ``apply_cells``  -- the local operator A: V_cell -> V_cell^* (Section 3.1):
  y_K = A_K (mask x_K) per cell with boundary copies of y set to zero.  Its
  scatter is ``apply_global`` of any x whose gather it was applied to.
* ``diagonal`` -- the diagonal d of the assembled A_CG, the vector the Jacobi
  preconditioner of Section 3.3 scales by: the diagonal of
  sum_K G_K^T A_K G_K is sum_K G_K^T diag(A_K), each A_K by plain quadrature.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .element import element_mass, element_stiffness, reference_directional
from .mesh import Mesh


def gather(mesh: Mesh, x: np.ndarray) -> np.ndarray:
    return np.asarray(x)[mesh.dofs]


def scatter(mesh: Mesh, y_cells: np.ndarray) -> np.ndarray:
    return np.bincount(mesh.dofs.ravel(), weights=np.asarray(y_cells).ravel(),
                       minlength=mesh.nglob)


def dss(mesh: Mesh, v_cells: np.ndarray) -> np.ndarray:
    return gather(mesh, scatter(mesh, v_cells))


def boundary_copies(mesh: Mesh) -> np.ndarray:
    """Boolean [ncells, n1^3]: copies that sit on the domain boundary."""
    return mesh.boundary_mask()[mesh.dofs]


def _cell_coefficients(mesh: Mesh, cells=None):
    hx, hy, hz = mesh.cell_sizes(cells)
    return hy * hz / hx, hx * hz / hy, hx * hy / hz


def apply_cells(mesh: Mesh, x_cells: np.ndarray, dirichlet: bool = True,
                cells=None) -> np.ndarray:
    """Local Laplace apply on cell-wise data (rows of ``x_cells`` are cells)."""
    Ax, Ay, Az, _ = reference_directional(mesh.p)
    X = np.array(x_cells, dtype=float, copy=True)
    if cells is None:
        cells = np.arange(mesh.ncells)
    if dirichlet:
        bmask = mesh.boundary_mask()[mesh.cell_dofs(cells)]
        X[bmask] = 0.0
    cx, cy, cz = _cell_coefficients(mesh, cells)
    Y = cx[:, None] * (X @ Ax) + cy[:, None] * (X @ Ay) + cz[:, None] * (X @ Az)
    if dirichlet:
        Y[bmask] = 0.0
    return Y


def mass_cells(mesh: Mesh, x_cells: np.ndarray, dirichlet: bool = True,
               cells=None) -> np.ndarray:
    """Local mass apply on cell-wise data (boundary copies of y zeroed)."""
    _, _, _, M = reference_directional(mesh.p)
    if cells is None:
        cells = np.arange(mesh.ncells)
    hx, hy, hz = mesh.cell_sizes(cells)
    Y = (hx * hy * hz)[:, None] * (np.asarray(x_cells, dtype=float) @ M)
    if dirichlet:
        Y[mesh.boundary_mask()[mesh.cell_dofs(cells)]] = 0.0
    return Y


def apply_global(mesh: Mesh, x: np.ndarray, dirichlet: bool = True) -> np.ndarray:
    """y = A_D x (or A_CG x when ``dirichlet`` is False), matrix-free."""
    return scatter(mesh, apply_cells(mesh, gather(mesh, x), dirichlet))


def mass_global(mesh: Mesh, x: np.ndarray, dirichlet: bool = True) -> np.ndarray:
    """y = P_I M_CG x (or M_CG x), matrix-free."""
    return scatter(mesh, mass_cells(mesh, gather(mesh, x), dirichlet))


def diagonal(mesh: Mesh) -> np.ndarray:
    """Diagonal of the assembled (Neumann) A_CG, summed from element diagonals."""
    hx, hy, hz = mesh.cell_sizes()
    cache = {}
    dcell = np.empty((mesh.ncells, mesh.n1 ** 3))
    for e in range(mesh.ncells):
        key = (hx[e], hy[e], hz[e])
        if key not in cache:
            cache[key] = np.diag(element_stiffness(mesh.p, *key)).copy()
        dcell[e] = cache[key]
    return scatter(mesh, dcell)


def assemble(mesh: Mesh, kind: str = "stiffness", dirichlet: bool = False):
    """Sparse global matrix sum_K G_K^T A_K G_K, each A_K by plain quadrature.

    With ``dirichlet`` the boundary rows and columns are zeroed (A_D).  Meant
    for small meshes: it builds one element matrix per distinct cell size.
    """
    n1c = mesh.n1 ** 3
    hx, hy, hz = mesh.cell_sizes()
    fn = element_stiffness if kind == "stiffness" else element_mass
    cache = {}
    rows, cols, vals = [], [], []
    dofs = mesh.dofs
    for e in range(mesh.ncells):
        key = (hx[e], hy[e], hz[e])
        if key not in cache:
            cache[key] = fn(mesh.p, *key)
        Ae = cache[key]
        rows.append(np.repeat(dofs[e], n1c))
        cols.append(np.tile(dofs[e], n1c))
        vals.append(Ae.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(mesh.nglob, mesh.nglob)).tocsr()
    if dirichlet:
        keep = sp.diags((~mesh.boundary_mask()).astype(float))
        A = (keep @ A @ keep).tocsr()
    return A
