"""Smoother and (flexible) PCG on assembled global vectors (oracle).

* ``smoother``: nu sweeps of damped Richardson on additive Schwarz starting
  from zero,  z_0 = 0,  z_{j+1} = z_j + omega * P_AS (r - A_D z_j).  The paper
  names overlapping Schwarz patch smoothers but gives no damping or sweep
  count; this is the reading the repository documents (omega = 1/8, two
  sweeps by default).
* ``dss_preconditioner`` and ``jacobi``: the simple preconditioners of
  Section 3.3 on assembled vectors.  P = S = G I_Riesz G^T is, in the
  assembled space, the Riesz identity: the assembled residual read as nodal
  values.  The Jacobi variant scales it by the inverse diagonal of A_CG
  (Eq. "dss_operator" and the identity G D_CG^{-1} = D_cell^{-1} G after it).
  With homogeneous Dirichlet conditions both act on the interior nodes only
  (the boundary rows of A_D are zero, so its boundary diagonal is empty).
* ``fcg``: the paper's Algorithm "Communication-Free (F)PCG" (Section 3.2),
  run on the assembled system A_CG u = b_CG.  By the equivalence theorem of
  that section the cell-wise iteration produces u_k = G u_k^global, so these
  iterates are what the device solve must reproduce.  The step length is the
  pairing quotient <r_k, z_k> / <q_k, p_k>; beta is <r_{k+1}, z_{k+1}> /
  <r_k, z_k> for the static (PCG) variant and -<q_k, z_{k+1}> / <q_k, p_k> for
  the flexible (FCG) variant.  The paper leaves the stopping test open; the
  reading here is the assembled relative residual ||r_k||_2 <= rtol ||b||_2 on
  the recursively updated residual.
"""
from __future__ import annotations

import numpy as np

from .mesh import Mesh
from .operators import apply_global, diagonal
from .patches import SchwarzFactors, additive_schwarz


def smoother(mesh: Mesh, r: np.ndarray, sweeps: int = 2, omega: float = 0.125,
             schwarz=None) -> np.ndarray:
    if schwarz is None:
        def schwarz(v):
            return additive_schwarz(mesh, v)
    z = np.zeros_like(r)
    for _ in range(sweeps):
        z = z + omega * schwarz(r - apply_global(mesh, z))
    return z


def dss_preconditioner(mesh: Mesh, r: np.ndarray) -> np.ndarray:
    """P r for P = S: the assembled residual as nodal values (interior only)."""
    return np.where(mesh.boundary_mask(), 0.0, r)


def jacobi(mesh: Mesh, r: np.ndarray, diag=None) -> np.ndarray:
    """P r for P = D_CG^{-1} S: the assembled residual divided by the
    diagonal of the assembled operator (interior only)."""
    d = diagonal(mesh) if diag is None else diag
    out = np.zeros_like(r)
    inner = ~mesh.boundary_mask()
    out[inner] = r[inner] / d[inner]
    return out


def fcg(apply, precond, b: np.ndarray, u0=None, rtol: float = 1e-8, maxit: int = 1000,
        variant: str = "fcg", record: bool = False):
    """(F)PCG on global vectors. Returns (u, iters, relres_history, iterates)."""
    u = np.zeros_like(b) if u0 is None else np.array(u0, dtype=float)
    r = b - apply(u)
    z = precond(r)
    p = z.copy()
    bnorm = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / bnorm]
    iterates = [u.copy()] if record else None
    rz = float(r @ z)
    k = 0
    while k < maxit:
        if hist[-1] <= rtol:
            break
        q = apply(p)
        qp = float(q @ p)
        alpha = rz / qp
        u = u + alpha * p
        r = r - alpha * q
        k += 1
        hist.append(np.linalg.norm(r) / bnorm)
        if record:
            iterates.append(u.copy())
        if hist[-1] <= rtol:
            break
        z = precond(r)
        if variant == "pcg":
            rz_new = float(r @ z)
            beta = rz_new / rz
        else:
            beta = -float(q @ z) / qp
            rz_new = float(r @ z)
        rz = rz_new
        p = z + beta * p
    return u, k, hist, iterates


def solve_poisson(mesh: Mesh, b: np.ndarray, rtol: float = 1e-8, maxit: int = 1000,
                  sweeps: int = 2, omega: float = 0.125, variant: str = "pcg",
                  record: bool = False, precond: str = "schwarz"):
    """FCG/PCG on A_D u = b preconditioned by the Schwarz smoother (or, with
    ``precond`` "dss" or "jacobi", by the simple preconditioners)."""
    def apply(v):
        return apply_global(mesh, v)

    if precond == "schwarz":
        factors = SchwarzFactors(mesh)

        def precond_fn(v):
            return smoother(mesh, v, sweeps, omega, schwarz=factors)
    elif precond == "dss":
        def precond_fn(v):
            return dss_preconditioner(mesh, v)
    elif precond == "jacobi":
        d = diagonal(mesh)

        def precond_fn(v):
            return jacobi(mesh, v, d)
    else:
        raise ValueError(precond)
    return fcg(apply, precond_fn, b, rtol=rtol, maxit=maxit, variant=variant, record=record)

