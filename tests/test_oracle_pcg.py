"""Pins of the oracle's PCG: finite termination of CG, exact preconditioning
and convergence with the HIF-DE preconditioner (Section 5)."""
import numpy as np
import scipy.sparse as sp

from oracle import hifde as OH
from oracle import pcg as OP
from synth import workloads as W


def test_cg_finite_termination():
    """CG on an SPD matrix with k distinct eigenvalues terminates in k steps."""
    ev = np.repeat([1.0, 3.0, 7.0, 20.0], 25)
    A = sp.diags(ev)
    f = np.random.default_rng(0).standard_normal(ev.size)
    x, it, rr = OP.pcg(A, f, lambda r: r, tol=1e-12, maxit=50)
    assert it <= 4 and rr <= 1e-12


def test_exact_preconditioner_one_step():
    a = W.make_field(2, 32, "loguniform", 1)
    F = OH.factor(2, 32, 4, a, eps=0.0)
    f = np.random.default_rng(1).standard_normal(F.N)
    x, it, rr = OP.pcg(F.A, f, lambda r: OH.solve(F, r), tol=1e-12, maxit=10)
    assert it == 1 and rr <= 1e-12


def test_hifde_preconditioner_converges():
    a = W.make_field(2, 64, "bernoulli_contrast", 2)
    F = OH.factor(2, 64, 8, a, eps=1e-6)
    f = W.make_rhs(F.N, 2, 3)
    for flexible in (False, True):
        X, its, rr = OP.pcg_multi(F.A, f, lambda r: OH.solve(F, r), 1e-12, 100, flexible)
        assert np.all(rr <= 2e-12) and np.all(its <= 19)


def test_flexible_equals_standard_with_symmetric_preconditioner():
    """With a symmetric preconditioner r_new^T z_old = 0 in exact arithmetic
    (the preconditioned residuals are conjugate), so the flexible update is
    the standard one: same iteration counts, same iterates to rounding."""
    a = W.make_field(2, 32, "loguniform", 4)
    F = OH.factor(2, 32, 4, a, eps=1e-4)
    f = W.make_rhs(F.N, 2, 5)
    Xs, its_s, _ = OP.pcg_multi(F.A, f, lambda r: OH.solve(F, r), 1e-12, 100, False)
    Xf, its_f, _ = OP.pcg_multi(F.A, f, lambda r: OH.solve(F, r), 1e-12, 100, True)
    assert np.array_equal(its_s, its_f)
    assert np.max(np.abs(Xs - Xf)) <= 1e-10 * np.max(np.abs(Xs))


def test_flexible_converges_with_nonsymmetric_preconditioner():
    """A preconditioner that is not symmetric (F^-1 followed by a small
    skew perturbation): the flexible variant still reaches the solution of a
    sparse direct solve."""
    import scipy.sparse.linalg as spla
    a = W.make_field(2, 32, "loguniform", 6)
    F = OH.factor(2, 32, 4, a, eps=1e-4)
    rng = np.random.default_rng(7)
    S = rng.standard_normal((F.N, 8))
    K = 1e-3 * (S[:, :4] @ S[:, 4:].T - S[:, 4:] @ S[:, :4].T) / F.N

    def prec(r):
        z = OH.solve(F, r)
        return z + K @ z

    f = W.make_rhs(F.N, 1, 8)[:, 0]
    z1, z2 = prec(f), prec(f[::-1].copy())
    assert abs(f[::-1] @ z1 - f @ z2) > 1e-12 * abs(f @ z1)      # really not symmetric
    x, it, rr = OP.pcg(F.A, f, prec, 1e-12, 200, flexible=True)
    xd = spla.spsolve(F.A.tocsc(), f)
    assert rr <= 2e-12
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
