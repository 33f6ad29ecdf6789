"""Element matrices by plain 3D quadrature (oracle; test infrastructure).

The Laplace element matrix of an axis-aligned box of sizes (hx, hy, hz) is

    A_K[alpha, beta] = sum_q w_q |J| grad(phi_alpha)(x_q) . grad(phi_beta)(x_q)

with phi_alpha(x, y, z) = l_a(xi) l_b(eta) l_c(zeta) the tensor-product
Lagrange basis on GLL nodes, the (p+1)^3-point Gauss rule, |J| = hx hy hz and
d/dx = (1/hx) d/dxi on the box.  This is the bilinear form of the Poisson
problem written out point by point; it does not use the Kronecker
factorisation of the operator (Eq. of Section 2.3), which the tests check
against it instead.  The mass matrix is the same sum with phi_alpha phi_beta.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from .basis import gauss_rule, gll_nodes, lagrange_derivs, lagrange_values


@lru_cache(maxsize=16)
def _point_tables(p: int):
    """Basis values and reference gradients at every 3D quadrature point.

    Returns (W, Phi, Gxi, Geta, Gzeta), Phi[q, alpha] etc., with quadrature
    point q = qx + nq (qy + nq qz) and basis alpha = a + n1 (b + n1 c).
    """
    xi = gll_nodes(p)
    nq = p + 1
    xq, wq = gauss_rule(nq)
    V = lagrange_values(xi, xq)      # V[q1, a]
    D = lagrange_derivs(xi, xq)      # D[q1, a]
    n1 = p + 1
    qx, qy, qz = np.meshgrid(np.arange(nq), np.arange(nq), np.arange(nq), indexing="ij")
    qx, qy, qz = qx.transpose(2, 1, 0).ravel(), qy.transpose(2, 1, 0).ravel(), qz.transpose(2, 1, 0).ravel()
    a = np.arange(n1 ** 3) % n1
    b = (np.arange(n1 ** 3) // n1) % n1
    c = np.arange(n1 ** 3) // (n1 * n1)
    W = wq[qx] * wq[qy] * wq[qz]
    Phi = V[qx][:, a] * V[qy][:, b] * V[qz][:, c]
    Gxi = D[qx][:, a] * V[qy][:, b] * V[qz][:, c]
    Geta = V[qx][:, a] * D[qy][:, b] * V[qz][:, c]
    Gzeta = V[qx][:, a] * V[qy][:, b] * D[qz][:, c]
    return W, Phi, Gxi, Geta, Gzeta


def element_stiffness(p: int, hx: float, hy: float, hz: float) -> np.ndarray:
    """Laplace element matrix of an hx x hy x hz box by plain quadrature."""
    W, _, Gxi, Geta, Gzeta = _point_tables(p)
    vol = hx * hy * hz
    Gx, Gy, Gz = Gxi / hx, Geta / hy, Gzeta / hz
    wv = W * vol
    return (Gx.T * wv) @ Gx + (Gy.T * wv) @ Gy + (Gz.T * wv) @ Gz


def element_mass(p: int, hx: float, hy: float, hz: float) -> np.ndarray:
    """Mass element matrix of an hx x hy x hz box by plain quadrature."""
    W, Phi, _, _, _ = _point_tables(p)
    return (Phi.T * (W * hx * hy * hz)) @ Phi


@lru_cache(maxsize=16)
def reference_directional(p: int):
    """Reference-box matrices  Ad[alpha,beta] = sum_q w_q d_d phi_alpha d_d phi_beta.

    For a box of sizes h, the change of variables gives
    A_K = (hy hz/hx) Ax + (hx hz/hy) Ay + (hx hy/hz) Az, which the oracle uses
    to apply many differently sized cells at once (a regrouping of the same
    quadrature sum, checked against ``element_stiffness`` by the tests).
    """
    W, Phi, Gxi, Geta, Gzeta = _point_tables(p)
    Ax = (Gxi.T * W) @ Gxi
    Ay = (Geta.T * W) @ Geta
    Az = (Gzeta.T * W) @ Gzeta
    M = (Phi.T * W) @ Phi
    return Ax, Ay, Az, M
