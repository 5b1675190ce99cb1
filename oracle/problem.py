"""Discretization of -div(a grad u) + b u = f on the unit square/cube.

Follows the five-point (2D, Section 3.1) and seven-point (3D, Section 3.2)
finite-difference stencils with the coefficient ``a`` sampled on the
staggered links and ``b`` at the nodes, homogeneous Dirichlet boundary
conditions, and ``h = 1/(n+1)`` for ``n`` unknowns per side (the paper writes
``N = (n-1)^d`` with ``h = 1/n``; here ``n`` counts unknowns).  A zero
coefficient on the boundary links of a side drops their Dirichlet term and
makes that side zero-flux (Neumann, first order): mixed boundary conditions
(Section 6) without a change of stencil.

Pinned by: the DST-I closed-form eigen-decomposition of the constant
coefficient Laplacian (tests/test_oracle_problem.py), brute-force assembly
at n <= 4, symmetry, and the closed-form spectrum of a grid with one
zero-flux side.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def dof_coords(dim: int, n: int) -> np.ndarray:
    """``(N, dim)`` integer coordinates; column k is x_k, x0 fastest."""
    idx = np.arange(n ** dim)
    return np.stack([(idx // n ** k) % n for k in range(dim)], axis=1)


def link_value(a_k: np.ndarray, dim: int, n: int, k: int, coords: np.ndarray,
               j: np.ndarray) -> np.ndarray:
    """Value of link ``j`` along axis ``k`` at the transverse coordinates of
    ``coords`` (the k-th coordinate of ``coords`` is ignored)."""
    idx = []
    for pos in range(dim):
        axis = dim - 1 - pos
        idx.append(j if axis == k else coords[:, axis])
    return a_k[tuple(idx)]


def assemble(dim: int, n: int, a, b=None) -> sp.csr_matrix:
    """Sparse symmetric A with rows
    ``A_ii = h^-2 sum_k (a_k[x_k] + a_k[x_k+1]) + b_i`` and
    ``A_{i, i+e_k} = -h^-2 a_k[x_k+1]`` (the link between x_k and x_k+1)."""
    N = n ** dim
    h2inv = float(n + 1) ** 2
    X = dof_coords(dim, n)
    idx = np.arange(N)
    rows, cols, vals = [], [], []
    diag = np.zeros(N) if b is None else np.asarray(b, dtype=np.float64).reshape(N).copy()
    for k in range(dim):
        lo = link_value(a[k], dim, n, k, X, X[:, k])        # link x_k   (to x_k-1)
        hi = link_value(a[k], dim, n, k, X, X[:, k] + 1)    # link x_k+1 (to x_k+1)
        diag += h2inv * (lo + hi)
        has_up = X[:, k] < n - 1
        i = idx[has_up]
        jn = i + n ** k
        v = -h2inv * hi[has_up]
        rows += [i, jn]
        cols += [jn, i]
        vals += [v, v]
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def stencil_pattern(A: sp.csr_matrix) -> sp.csr_matrix:
    """Structural pattern of A as a 0/1 matrix (entries are never dropped)."""
    P = A.copy().tocsr()
    P.data = np.ones_like(P.data)
    return P
