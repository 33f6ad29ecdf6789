"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random numbers and builds workload descriptions; it
holds none of the finite-element arithmetic.  Every workload is a Cartesian
tensor-product hexahedral mesh of the unit cube, the mesh family the paper
benchmarks on (Section 6, uniform refinement of the unit cube).

Conventions (fixed here once so that both sides of every comparison draw the
same numbers):

* generator: ``numpy.random.default_rng(seed)`` (PCG64);
* cell widths are drawn first, x then y then z, each ``uniform(0.5, 1.5, n)``
  and renormalised to sum to one (a graded tensor mesh of the unit cube);
* vectors over global nodes are drawn next from the same generator, in
  lexicographic global order with x fastest:
  ``g = I + (n_x p + 1) * (J + (n_y p + 1) * K)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload", "graded_widths", "uniform_widths", "global_len",
    "workload_apply_q2_small", "workload_q3_graded", "workload_q2_graded",
    "workload_q7_graded", "batch_problems", "serve_stream",
]


def global_len(p: int, n) -> int:
    n = _n3(n)
    return (n[0] * p + 1) * (n[1] * p + 1) * (n[2] * p + 1)


def _n3(n):
    if isinstance(n, (int, np.integer)):
        return (int(n),) * 3
    n = tuple(int(v) for v in n)
    assert len(n) == 3
    return n


def uniform_widths(n):
    n = _n3(n)
    return [np.full(nd, 1.0 / nd) for nd in n]


def graded_widths(rng: np.random.Generator, n):
    """Per-direction widths uniform[0.5, 1.5], renormalised to the unit cube."""
    n = _n3(n)
    out = []
    for nd in n:
        w = rng.uniform(0.5, 1.5, nd)
        out.append(w / w.sum())
    return out


@dataclass
class Workload:
    """One synthetic Poisson problem: mesh description plus a seeded vector."""
    name: str
    p: int
    n: tuple
    widths: list
    x: np.ndarray               # vector over global nodes (len = global_len)
    noise: np.ndarray | None = None   # N(0,1) draws for a noisy right-hand side
    meta: dict = field(default_factory=dict)


def workload_apply_q2_small(seed: int = 0) -> Workload:
    """Q2, 8^3 uniform cells (4913 nodes), x ~ U[-1,1] from ``seed``."""
    p, n = 2, (8, 8, 8)
    rng = np.random.default_rng(seed)
    w = uniform_widths(n)
    x = rng.uniform(-1.0, 1.0, global_len(p, n))
    return Workload("q2_8cubed_uniform", p, n, w, x)


def _graded(name, p, nc, seed, noise_seed=None):
    n = _n3(nc)
    rng = np.random.default_rng(seed)
    w = graded_widths(rng, n)
    x = rng.uniform(-1.0, 1.0, global_len(p, n))
    noise = None
    if noise_seed is not None:
        noise = np.random.default_rng(noise_seed).standard_normal(global_len(p, n))
    return Workload(name, p, n, w, x, noise)


def workload_q3_graded(nc: int = 64, seed: int = 1) -> Workload:
    """Q3 on an nc^3 graded mesh (64^3 -> 193^3 nodes), x ~ U[-1,1]."""
    return _graded(f"q3_{nc}cubed_graded", 3, nc, seed)


def workload_q2_graded(nc: int = 96, seed: int = 1) -> Workload:
    """Q2 on an nc^3 graded mesh (96^3 -> 193^3 nodes, same node count as Q3 64^3)."""
    return _graded(f"q2_{nc}cubed_graded", 2, nc, seed)


def workload_q7_graded(nc: int = 24, seed: int = 1, noise_seed: int = 2) -> Workload:
    """Q7 on an nc^3 graded mesh (24^3 -> 169^3 nodes); widths from ``seed``,
    right-hand-side noise N(0,1) from ``noise_seed``."""
    return _graded(f"q7_{nc}cubed_graded", 7, nc, seed, noise_seed)


def batch_problems(count: int = 256, seed: int = 3, degrees=(2, 3, 7),
                   nmin: int = 4, nmax: int = 32):
    """Independent problems for one batched launch: degree uniform from
    ``degrees``, n uniform integer in [nmin, nmax], uniform cube mesh, and a
    vector x ~ U[-1,1] per problem (drawn in problem order)."""
    rng = np.random.default_rng(seed)
    ps = rng.choice(np.asarray(degrees), size=count)
    ns = rng.integers(nmin, nmax + 1, size=count)
    out = []
    for i in range(count):
        p, nc = int(ps[i]), int(ns[i])
        n = (nc, nc, nc)
        x = rng.uniform(-1.0, 1.0, global_len(p, n))
        out.append(Workload(f"batch{i}_q{p}_{nc}", p, n, uniform_widths(n), x))
    return out


def serve_stream(count: int = 10000, rate: float = 200.0, seed: int = 4,
                 degrees=(2, 3, 7), weights=(0.4, 0.4, 0.2),
                 median_n: float = 12.0, sigma: float = 0.5,
                 nmin: int = 4, nmax: int = 48):
    """Request stream for the serving loop.

    Returns a list of dicts with ``t`` (arrival time in seconds, Poisson
    process of the given rate), ``p``, ``n`` (cells per direction, lognormal
    with the given median and log-space sigma, rounded and clipped) and
    ``seed`` (per-request seed for its right-hand side).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    ps = rng.choice(np.asarray(degrees), size=count, p=np.asarray(weights))
    ns = np.rint(np.exp(math.log(median_n) + sigma * rng.standard_normal(count)))
    ns = np.clip(ns, nmin, nmax).astype(int)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    return [dict(t=float(t[i]), p=int(ps[i]), n=int(ns[i]), seed=int(seeds[i]))
            for i in range(count)]


def request_rhs_nodal(p: int, n, seed: int) -> np.ndarray:
    """Nodal source values f ~ U[-1,1] over global nodes for one request."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, global_len(p, n))
