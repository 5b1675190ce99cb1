"""Restarted GMRES with right preconditioning (the Krylov solver the paper
pairs with the factorization for indefinite problems, Section 5).

For A x = f from x0 = 0: with z = M r the Arnoldi process builds an
orthonormal basis V of the Krylov space of A M (modified Gram-Schmidt), the
Hessenberg least-squares problem is solved by Givens rotations, and
x = x0 + M V y.  It restarts every ``restart`` steps, stops when the
residual estimate falls to ``tol ||f||`` or after ``maxit`` steps, and
reports the true residual.  Columns of a multi-column right-hand side are
independent.

Pinned by: each step's residual equals the minimum over the Krylov space
computed by a direct least-squares solve; an exact preconditioner gives the
solution in one step; convergence to a sparse direct solution of an
indefinite Helmholtz-type system (tests/test_oracle_gmres.py).
"""
from __future__ import annotations

import numpy as np


def gmres(A, f: np.ndarray, precond, tol: float = 1e-12, restart: int = 30,
          maxit: int = 300, history: bool = False):
    """Returns ``(x, iters, relres_true)`` (and the residual estimates of
    every step when ``history``)."""
    f = np.asarray(f, dtype=np.float64)
    N = f.shape[0]
    nf = np.linalg.norm(f)
    x = np.zeros(N)
    hist = []
    if nf == 0.0:
        return (x, 0, 0.0, hist) if history else (x, 0, 0.0)
    it = 0
    while it < maxit:
        r = f - A @ x
        beta = np.linalg.norm(r)
        if beta <= tol * nf:
            break
        V = np.zeros((N, restart + 1))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[:, 0] = r / beta
        k_done = 0
        for k in range(restart):
            it += 1
            w = A @ precond(V[:, k])
            for i in range(k + 1):
                H[i, k] = V[:, i] @ w
                w = w - H[i, k] * V[:, i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] > 0.0:
                V[:, k + 1] = w / H[k + 1, k]
            for i in range(k):   # earlier rotations on the new column
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            rho = np.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = H[k, k] / rho, H[k + 1, k] / rho
            H[k, k], H[k + 1, k] = rho, 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            hist.append(abs(g[k + 1]) / nf)
            k_done = k + 1
            if abs(g[k + 1]) <= tol * nf or it >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:k_done, :k_done]), g[:k_done])
        x = x + precond(V[:, :k_done] @ y)
        if abs(g[k_done]) <= tol * nf:
            break
    relres = float(np.linalg.norm(f - A @ x) / nf)
    return (x, it, relres, hist) if history else (x, it, relres)


def gmres_multi(A, F: np.ndarray, precond, tol=1e-12, restart=30, maxit=300):
    """Column-by-column GMRES; returns ``(X, iters[], relres[])``."""
    X = np.zeros_like(F, dtype=np.float64)
    its, res = [], []
    for j in range(F.shape[1]):
        x, it, rr = gmres(A, F[:, j], precond, tol, restart, maxit)
        X[:, j] = x
        its.append(it)
        res.append(rr)
    return X, np.array(its), np.array(res)
