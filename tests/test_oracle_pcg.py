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
