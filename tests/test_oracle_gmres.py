"""Pins of the oracle's indefinite factorization (unpivoted LDL^T with
negative pivots) and of its restarted GMRES (Section 5: indefinite problems
with the factorization as preconditioner)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import gmres as OG
from oracle import hifde as OH
from oracle import problem
from synth import workloads as W

# Helmholtz-type problem: a = 1, b = -60 on the 32^2 grid (h = 1/33).  The
# Laplacian's eigenvalues 4 h^-2 (sin^2(j pi h/2) + sin^2(k pi h/2)) are
# 19.7, 49.2 (twice), 78.7, ...: A has three negative eigenvalues, while the
# 7 x 7 interiors of the 8 x 8 leaf cells (smallest eigenvalue about 330)
# stay positive definite.
N2, LEAF, BNEG = 32, 8, -60.0


def _helmholtz():
    a = W.make_field(2, N2, "const", None)
    b = np.full(N2 * N2, BNEG)
    return a, b, problem.assemble(2, N2, a, b)


def test_ldl_sym_reconstructs_and_keeps_inertia():
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    ev = np.concatenate([-np.geomspace(1, 50, 7), np.geomspace(1, 80, 33)])
    A = (Q * ev) @ Q.T
    L, D = OH.ldl_sym(A)
    assert np.allclose(np.tril(L), L) and np.allclose(np.diag(L), 1.0)
    assert np.max(np.abs(L @ np.diag(D) @ L.T - A)) <= 1e-10 * np.max(np.abs(A))
    # Sylvester's law of inertia: A = L D L^T is a congruence
    assert np.sum(D < 0) == 7


def test_ldl_sym_equals_cholesky_form_on_spd():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((30, 30))
    A = X @ X.T + 30 * np.eye(30)
    L1, D1 = OH.ldl_sym(A)
    L2, D2 = OH.ldl_spd(A)
    assert np.allclose(L1, L2, atol=1e-12) and np.allclose(D1, D2, rtol=1e-12)


def test_ldl_sym_reports_breakdown():
    A = np.array([[1.0, 1.0], [1.0, 1.0]])       # second pivot exactly 0
    with pytest.raises(OH.Breakdown):
        OH.ldl_sym(A)


def test_gmres_steps_minimize_over_the_krylov_space():
    """Without restart and with M = I, step k's residual is the minimum of
    ||f - A y|| over the k-dimensional Krylov space (brute force: an
    orthonormal basis of [f, A f, ..., A^{k-1} f] and a least-squares solve)."""
    rng = np.random.default_rng(2)
    n = 40
    A = rng.standard_normal((n, n)) + 8 * np.eye(n)
    f = rng.standard_normal(n)
    _, _, _, hist = OG.gmres(A, f, lambda r: r, tol=1e-14, restart=n, maxit=12, history=True)
    K = np.zeros((n, 12))
    v = f.copy()
    for k in range(12):
        K[:, k] = v
        v = A @ v
    for k in range(1, 13):
        Qk, _ = np.linalg.qr(K[:, :k])
        y = np.linalg.lstsq(A @ Qk, f, rcond=None)[0]
        best = np.linalg.norm(f - A @ Qk @ y) / np.linalg.norm(f)
        assert hist[k - 1] == pytest.approx(best, rel=1e-8, abs=1e-14), k


def test_exact_indefinite_factorization_is_a_direct_solve():
    """eps = 0 is the multifrontal method: F = A, so F^-1 f is the sparse
    direct solution, GMRES takes one step, and the pivots of D carry A's
    inertia (three negative eigenvalues)."""
    a, b, A = _helmholtz()
    ev = np.linalg.eigvalsh(A.toarray())
    assert np.sum(ev < 0) == 3
    F = OH.factor(2, N2, LEAF, a, b=b, eps=0.0, definite=False)
    f = W.make_rhs(N2 * N2, 1, 3)[:, 0]
    ud = spla.spsolve(A.tocsc(), f)
    u = OH.solve(F, f)
    assert np.linalg.norm(u - ud) <= 1e-12 * np.linalg.norm(ud)
    D = np.concatenate([c.D for lev in F.levels for c in lev.cells] + [F.top.D])
    assert np.sum(D < 0) == 3
    x, it, rr = OG.gmres(A, f, lambda r: OH.solve(F, r), 1e-12, 30, 50)
    assert it == 1 and rr <= 1e-12


@pytest.mark.parametrize("eps", [1e-6, 1e-3])
def test_indefinite_hifde_preconditioned_gmres(eps):
    a, b, A = _helmholtz()
    F = OH.factor(2, N2, LEAF, a, b=b, eps=eps, definite=False)
    f = W.make_rhs(N2 * N2, 2, 4)
    X, its, rr = OG.gmres_multi(A, f, lambda r: OH.solve(F, r), 1e-12, 30, 100)
    Xd = spla.spsolve(A.tocsc(), f)
    assert np.all(rr <= 1e-12), rr
    assert np.all(its <= 10), its
    assert np.linalg.norm(X - Xd) <= 1e-9 * np.linalg.norm(Xd)
    # the definite path refuses the same problem
    with pytest.raises(OH.NotSPD):
        OH.factor(2, N2, LEAF, a, b=b, eps=eps)
