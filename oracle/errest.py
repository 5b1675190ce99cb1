"""A posteriori error estimates of Section 5 by power iteration.

``e_a ~ ||A - F|| / ||A||`` and ``e_s ~ ||I - A F^{-1}||``, each by power
iteration from a uniform random start vector, stopped when the norm estimate
changes by less than a relative 1e-2 (capped at ``maxit`` steps).

Pinned by: dense ``numpy.linalg.norm(., 2)`` on small grids
(tests/test_oracle_hifde.py).
"""
from __future__ import annotations

import numpy as np


def power_norm(op, opT, n: int, seed: int = 0, rtol: float = 1e-2, maxit: int = 100) -> float:
    """Estimate ``||M||_2`` by power iteration on ``M^T M``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(0.0, 1.0, n)
    x /= np.linalg.norm(x)
    est = 0.0
    for _ in range(maxit):
        y = op(x)
        new = float(np.linalg.norm(y))
        z = opT(y)
        nz = np.linalg.norm(z)
        if nz == 0.0:
            return new
        x = z / nz
        if est > 0 and abs(new - est) <= rtol * new:
            return new
        est = new
    return est


def e_a(A, apply_F, seed=0, rtol=1e-2, maxit=100) -> float:
    n = A.shape[0]
    op = lambda v: A @ v - apply_F(v)
    nA = power_norm(lambda v: A @ v, lambda v: A @ v, n, seed, rtol, maxit)
    return power_norm(op, op, n, seed, rtol, maxit) / nA


def e_s(A, solve_F, seed=0, rtol=1e-2, maxit=100) -> float:
    n = A.shape[0]
    op = lambda v: v - A @ solve_F(v)
    opT = lambda v: v - solve_F(A @ v)
    return power_norm(op, opT, n, seed, rtol, maxit)
