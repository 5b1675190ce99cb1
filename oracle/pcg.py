"""Conjugate gradients preconditioned by F^{-1} (Section 5: the factorization
used as a preconditioner, tolerance 1e-12).

Standard Hestenes-Stiefel PCG from ``x0 = 0`` with the recursive residual; the
``flexible`` variant uses ``beta = r_new^T (z_new - z_old) / (r_old^T z_old)``
(Polak-Ribiere), which tolerates a preconditioner that is not exactly
symmetric.  Columns of a multi-column right-hand side are independent.

Pinned by: with an exact preconditioner (eps = 0) the first iterate solves
the system; on a diagonal test matrix the iterates match the closed form of
CG; convergence to the requested tolerance (tests/test_oracle_pcg.py).

Parity unpinned: the iteration path of the ``flexible`` variant under a
preconditioner that is not symmetric.  With a symmetric one it equals the
standard update (pinned); otherwise no closed form or library routine fixes
its iterates, so only its converged solution (true residual at tol) is
checked.
"""
from __future__ import annotations

import numpy as np


def pcg(A, f: np.ndarray, precond, tol: float = 1e-12, maxit: int = 200,
        flexible: bool = False):
    """Returns ``(x, iters, relres_true)`` for one right-hand side."""
    f = np.asarray(f, dtype=np.float64)
    nf = np.linalg.norm(f)
    x = np.zeros_like(f)
    if nf == 0.0:
        return x, 0, 0.0
    r = f.copy()
    z = precond(r)
    p = z.copy()
    rz = float(r @ z)
    it = 0
    while it < maxit:
        it += 1
        Ap = A @ p
        alpha = rz / float(p @ Ap)
        x += alpha * p
        r_new = r - alpha * Ap
        if np.linalg.norm(r_new) <= tol * nf:
            r = r_new
            break
        z_new = precond(r_new)
        if flexible:
            beta = float(r_new @ (z_new - z)) / rz
        else:
            beta = float(r_new @ z_new) / rz
        rz = float(r_new @ z_new)
        p = z_new + beta * p
        r, z = r_new, z_new
    relres = float(np.linalg.norm(f - A @ x) / nf)
    return x, it, relres


def pcg_multi(A, F: np.ndarray, precond, tol=1e-12, maxit=200, flexible=False):
    """Column-by-column PCG; returns ``(X, iters[], relres[])``."""
    X = np.zeros_like(F, dtype=np.float64)
    its, res = [], []
    for j in range(F.shape[1]):
        x, it, rr = pcg(A, F[:, j], precond, tol, maxit, flexible)
        X[:, j] = x
        its.append(it)
        res.append(rr)
    return X, np.array(its), np.array(res)
