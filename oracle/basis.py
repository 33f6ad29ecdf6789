"""1D ingredients of the Q_p Lagrange element (oracle; test infrastructure).

The paper states the element only as "nodal values" with 1D mass and
derivative contractions (Section 2.3).  The reading taken here: Lagrange
polynomials on the p+1 Gauss-Lobatto-Legendre (GLL) nodes, integrated with the
(p+1)-point Gauss-Legendre rule, all on the reference interval [0, 1].
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as leg


def gll_nodes(p: int) -> np.ndarray:
    """GLL nodes on [0,1]: the end points plus the roots of P_p' (mapped).

    Roots come from the Legendre companion matrix and are polished by Newton
    steps on P_p' so they are accurate to rounding.
    """
    if p < 1:
        raise ValueError("p >= 1")
    if p == 1:
        return np.array([0.0, 1.0])
    c = np.zeros(p + 1)
    c[p] = 1.0
    d1 = leg.legder(c)
    d2 = leg.legder(d1)
    r = np.sort(np.real(leg.legroots(d1)))
    for _ in range(4):
        r = r - leg.legval(r, d1) / leg.legval(r, d2)
    s = np.concatenate(([-1.0], r, [1.0]))
    return 0.5 * (s + 1.0)


def gauss_rule(nq: int):
    """nq-point Gauss-Legendre rule mapped to [0,1] (points, weights)."""
    s, w = leg.leggauss(nq)
    return 0.5 * (s + 1.0), 0.5 * w


def lagrange_values(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """V[q, a] = l_a(x_q), l_a the Lagrange polynomial with l_a(node_b) = delta_ab."""
    x = np.asarray(x, dtype=float)
    n1 = len(nodes)
    V = np.ones((len(x), n1))
    for a in range(n1):
        for b in range(n1):
            if b != a:
                V[:, a] *= (x - nodes[b]) / (nodes[a] - nodes[b])
    return V


def lagrange_derivs(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """D[q, a] = l_a'(x_q), by the product rule on the product form of l_a."""
    x = np.asarray(x, dtype=float)
    n1 = len(nodes)
    D = np.zeros((len(x), n1))
    for a in range(n1):
        for m in range(n1):
            if m == a:
                continue
            term = np.full(len(x), 1.0 / (nodes[a] - nodes[m]))
            for b in range(n1):
                if b != a and b != m:
                    term *= (x - nodes[b]) / (nodes[a] - nodes[b])
            D[:, a] += term
    return D


def mass_1d(p: int, h: float = 1.0) -> np.ndarray:
    """1D element mass matrix on an interval of length h, Gauss rule p+1."""
    xi = gll_nodes(p)
    xq, wq = gauss_rule(p + 1)
    V = lagrange_values(xi, xq)
    return h * (V.T * wq) @ V


def stiffness_1d(p: int, h: float = 1.0) -> np.ndarray:
    """1D element stiffness matrix on an interval of length h, Gauss rule p+1."""
    xi = gll_nodes(p)
    xq, wq = gauss_rule(p + 1)
    D = lagrange_derivs(xi, xq)
    return (D.T * wq) @ D / h
