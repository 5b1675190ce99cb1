"""Indefinite problems on the GPU (Section 5, Example 3): the factorization with
HIFDE_INDEFINITE (negative pivots accepted) and GMRES with F^-1 as right
preconditioner, against the oracle's indefinite factorization and GMRES and
against sparse direct solutions of the assembled matrix.

Helmholtz-type inputs: a = 1, b = -k^2 constant, so the eigenvalues of A are
4 h^-2 (sin^2(j pi h / 2) + sin^2(l pi h / 2)) - k^2 in closed form (their
signs give the inertia each case states)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import gmres as OG
from oracle import hifde as OH
from oracle import problem
from synth import workloads as W

from _helpers import torch_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _negative_eigenvalues(n, bneg):
    h = 1.0 / (n + 1)
    lam = 4 / h ** 2 * np.sin(np.arange(1, n + 1) * np.pi * h / 2) ** 2
    return int(np.sum(lam[:, None] + lam[None, :] + bneg < 0))


def _problem(n, bneg):
    a = W.make_field(2, n, "const", None)
    b = np.full(n * n, bneg)
    return a, b, problem.assemble(2, n, a, b)


def _factor(n, m, a, b, eps, prec, flags=None):
    import paper_1307_2895_amd as H
    T = H.hifde_build_tree(2, n, m, 0)
    fl = H.HIFDE_INDEFINITE if flags is None else flags
    F = H.hifde_factor(T, torch_inputs(a), torch.from_numpy(b).cuda(), eps, prec, flags=fl)
    return T, F


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_exact_indefinite_factorization(prec):
    """eps = 0: F = A up to the factor's precision.  In double GMRES stops
    after one step at the sparse direct solution; the float sweeps take a few
    more.  (32^2 grid, b = -60: three negative eigenvalues.)"""
    import paper_1307_2895_amd as H
    n, m, bneg = 32, 8, -60.0
    assert _negative_eigenvalues(n, bneg) == 3
    a, b, A = _problem(n, bneg)
    f = W.make_rhs(n * n, 2, 3)
    ud = spla.spsolve(A.tocsc(), f)
    print(f"case exact prec={prec}", flush=True)
    T, F = _factor(n, m, a, b, 0.0, prec)
    fd = torch.from_numpy(f).cuda()
    z = H.hifde_solve(F, fd).cpu().numpy()
    err = np.linalg.norm(z - ud) / np.linalg.norm(ud)
    print("F^-1 f vs direct", err)
    assert err <= (1e-12 if prec == 0 else 1e-4)
    u, its, rel = H.hifde_gmres(F, fd, tol=1e-12, restart=30, maxit=50)
    u = u.cpu().numpy()
    print("iters", its, "relres", rel)
    assert np.all(rel <= 1e-12)
    assert np.all(its == 1) if prec == 0 else np.all(its <= 4)
    assert np.linalg.norm(u - ud) <= 1e-10 * np.linalg.norm(ud)
    F.free()


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("n,bneg,eps", [(64, -300.0, 1e-6), (64, -300.0, 1e-3),
                                        (128, -1000.0, 1e-6), (128, -1000.0, 1e-3)])
def test_gmres_matches_oracle(n, bneg, eps, prec):
    """Same problem, factorization and solver on both sides: the double
    factor takes the oracle's step counts (one more or fewer at most, where a
    residual estimate sits at the tolerance); the float sweeps at most twice
    as many plus two.  Solutions agree with the sparse direct one."""
    import paper_1307_2895_amd as H
    m = 8
    neg = _negative_eigenvalues(n, bneg)
    assert neg in (19, 71)
    a, b, A = _problem(n, bneg)
    f = W.make_rhs(n * n, 2, 7)
    OF = OH.factor(2, n, m, a, b=b, eps=eps, definite=False)
    _, oits, orel = OG.gmres_multi(A, f, lambda r: OH.solve(OF, r), 1e-12, 30, 100)
    ud = spla.spsolve(A.tocsc(), f)
    print(f"case n={n} b={bneg} eps={eps} prec={prec}", flush=True)
    T, F = _factor(n, m, a, b, eps, prec)
    u, its, rel = H.hifde_gmres(F, torch.from_numpy(f).cuda(), tol=1e-12, restart=30, maxit=100)
    u = u.cpu().numpy()
    true_rel = np.linalg.norm(f - A @ u, axis=0) / np.linalg.norm(f, axis=0)
    err = np.linalg.norm(u - ud) / np.linalg.norm(ud)
    print("oracle iters", oits, "gpu iters", its, "relres", rel, "err", err)
    assert np.all(rel <= 1e-12), rel
    # both sides evaluate f - A u in double: about 1e-16 ||A|| ||u|| / ||f||
    # of noise apiece
    np.testing.assert_allclose(rel, true_rel, rtol=1e-2, atol=2e-15)
    if prec == 0:
        assert np.all(np.abs(its - oits) <= 1), (its, oits)
    else:
        assert np.all(its <= 2 * oits + 2), (its, oits)
    assert err <= 1e-8, err
    F.free()


def test_restarts_match_oracle():
    """restart = 2: every cycle after the first starts from the true
    residual; the step counts are the oracle's (double factor)."""
    import paper_1307_2895_amd as H
    n, m, bneg, eps = 64, 8, -300.0, 1e-3
    a, b, A = _problem(n, bneg)
    f = W.make_rhs(n * n, 3, 8)
    OF = OH.factor(2, n, m, a, b=b, eps=eps, definite=False)
    _, oits, _ = OG.gmres_multi(A, f, lambda r: OH.solve(OF, r), 1e-12, 2, 100)
    T, F = _factor(n, m, a, b, eps, H.HIFDE_FP64)
    u, its, rel = H.hifde_gmres(F, torch.from_numpy(f).cuda(), tol=1e-12, restart=2, maxit=100)
    print("oracle", oits, "gpu", its, rel)
    assert np.all(np.abs(its - oits) <= 1), (its, oits)
    assert np.all(rel <= 1e-12)
    ud = spla.spsolve(A.tocsc(), f)
    assert np.linalg.norm(u.cpu().numpy() - ud) <= 1e-9 * np.linalg.norm(ud)
    F.free()


@pytest.mark.parametrize("prec", [0, 2])
def test_one_step_is_the_minimal_residual_multiple(prec):
    """maxit = 1: u = alpha z with z = F^-1 f and alpha minimizing
    ||f - alpha A z|| (alpha = (A z . f) / (A z . A z)); ENOCONV with the
    outputs filled."""
    import paper_1307_2895_amd as H
    n, m, bneg, eps = 64, 8, -300.0, 1e-3
    a, b, A = _problem(n, bneg)
    f = W.make_rhs(n * n, 2, 9)
    T, F = _factor(n, m, a, b, eps, prec)
    fd = torch.from_numpy(f).cuda()
    with pytest.raises(H.HifdeError) as ei:
        H.hifde_gmres(F, fd, tol=1e-12, maxit=1)
    assert ei.value.code == H.HIFDE_ENOCONV
    u, its, rel = H.hifde_gmres(F, fd, tol=1e-12, maxit=1, raise_on_noconv=False)
    u = u.cpu().numpy()
    z = H.hifde_solve(F, fd).cpu().numpy()
    Az = A @ z
    alpha = np.sum(Az * f, axis=0) / np.sum(Az * Az, axis=0)
    assert np.all(its == 1)
    tol = 1e-9 if prec == 0 else 1e-5   # float sweeps: z rounded to float
    np.testing.assert_allclose(u, z * alpha, rtol=tol, atol=tol * np.abs(u).max())
    true_rel = np.linalg.norm(f - A @ u, axis=0) / np.linalg.norm(f, axis=0)
    np.testing.assert_allclose(rel, true_rel, rtol=1e-8)
    assert np.all(rel < 1.0) and np.all(rel > 1e-12)
    F.free()


def test_zero_column_and_argument_checks():
    import paper_1307_2895_amd as H
    n, m, bneg = 32, 8, -60.0
    a, b, A = _problem(n, bneg)
    f = W.make_rhs(n * n, 3, 10)
    f[:, 1] = 0.0
    T, F = _factor(n, m, a, b, 1e-6, H.HIFDE_FP64)
    fd = torch.from_numpy(f).cuda()
    u, its, rel = H.hifde_gmres(F, fd, tol=1e-12)
    u = u.cpu().numpy()
    assert its[1] == 0 and rel[1] == 0.0 and np.all(u[:, 1] == 0.0)
    assert np.all(rel <= 1e-12) and its[0] > 0 and its[2] > 0
    for kw in ({"restart": 0}, {"maxit": 0}, {"tol": 0.0}, {"tol": float("inf")},
               {"tol": float("nan")}):
        with pytest.raises(H.HifdeError) as ei:
            H.hifde_gmres(F, fd, **kw)
        assert ei.value.code == H.HIFDE_EINVAL, kw
    # conjugate gradients refuses an indefinite factor
    with pytest.raises(H.HifdeError) as ei:
        H.hifde_pcg(F, fd)
    assert ei.value.code == H.HIFDE_ESTATE
    F.free()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_indefinite_flag_on_a_definite_problem(prec):
    """With only positive pivots the flag changes no arithmetic: F^-1 is
    bitwise that of the definite factorization, and GMRES reaches the
    solution PCG finds."""
    import paper_1307_2895_amd as H
    n, m = 64, 8
    a = W.make_field(2, n, "bernoulli_contrast", 2)
    b = np.zeros(n * n)
    f = W.make_rhs(n * n, 2, 11)
    fd = torch.from_numpy(f).cuda()
    _, F1 = _factor(n, m, a, b, 1e-6, prec, flags=0)
    _, F2 = _factor(n, m, a, b, 1e-6, prec)
    z1 = H.hifde_solve(F1, fd).cpu().numpy()
    z2 = H.hifde_solve(F2, fd).cpu().numpy()
    assert np.array_equal(z1, z2)
    up, _, _ = H.hifde_pcg(F1, fd, tol=1e-12, maxit=100)
    ug, its, rel = H.hifde_gmres(F2, fd, tol=1e-12, maxit=100)
    print("gmres iters", its, rel)
    assert np.all(rel <= 1e-12)
    up, ug = up.cpu().numpy(), ug.cpu().numpy()
    assert np.linalg.norm(ug - up) <= 1e-8 * np.linalg.norm(up)
    F1.free()
    F2.free()


def test_indefinite_levels_fail_without_the_flag():
    """b = -1000 on the 128^2 grid keeps the level-0 blocks definite but not
    A: the definite factorization reports ENOTSPD, the indefinite one
    succeeds."""
    import paper_1307_2895_amd as H
    n, m, bneg = 128, 8, -1000.0
    a, b, _ = _problem(n, bneg)
    with pytest.raises(H.HifdeError) as ei:
        _factor(n, m, a, b, 1e-6, H.HIFDE_MIXED_ELIM64, flags=0)
    assert ei.value.code == H.HIFDE_ENOTSPD
    _, F = _factor(n, m, a, b, 1e-6, H.HIFDE_MIXED_ELIM64)
    F.free()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("eps,sketch", [(1e-6, False), (1e-3, False), (1e-6, True), (1e-3, True)])
def test_gmres_3d_matches_oracle(eps, sketch, prec):
    """The 3D analogue (Example 6) on the 16^3 grid at 8 unknowns per
    wavelength (kappa = 2: 17 negative eigenvalues, |lambda| >= 6.7 from the
    closed form), with and without the randomized ID on both sides."""
    import paper_1307_2895_amd as H
    n, m = 16, 4
    b = W.helmholtz_b(n ** 3, 2.0)
    a = W.make_field(3, n, "const", None)
    A = problem.assemble(3, n, a, b)
    f = W.make_rhs(n ** 3, 2, 7)
    OF = OH.factor(3, n, m, a, b=b, eps=eps, definite=False, sketch=sketch)
    _, oits, _ = OG.gmres_multi(A, f, lambda r: OH.solve(OF, r), 1e-12, 30, 100)
    ud = spla.spsolve(A.tocsc(), f)
    print(f"case 3d eps={eps} sketch={sketch} prec={prec}", flush=True)
    T = H.hifde_build_tree(3, n, m, 0)
    flags = H.HIFDE_INDEFINITE | (H.HIFDE_SKETCH_ID if sketch else 0)
    F = H.hifde_factor(T, torch_inputs(a), torch.from_numpy(b).cuda(), eps, prec, flags=flags)
    u, its, rel = H.hifde_gmres(F, torch.from_numpy(f).cuda(), tol=1e-12, maxit=100)
    u = u.cpu().numpy()
    err = np.linalg.norm(u - ud) / np.linalg.norm(ud)
    print("oracle iters", oits, "gpu iters", its, "relres", rel, "err", err)
    assert np.all(rel <= 1e-12)
    if prec == 0:
        assert np.all(np.abs(its - oits) <= 1), (its, oits)
    else:
        assert np.all(its <= 2 * oits + 2), (its, oits)
    assert err <= 1e-9
    F.free()


def test_gmres_many_columns():
    """300 right-hand sides (more than a work-group's threads: the inner
    products take the columns 256 at a time) on a small indefinite grid:
    every column converges to the sparse direct solution."""
    import paper_1307_2895_amd as H
    n, m, bneg = 32, 8, -60.0
    a, b, A = _problem(n, bneg)
    f = W.make_rhs(n * n, 300, 14)
    T, F = _factor(n, m, a, b, 1e-6, H.HIFDE_FP64)
    u, its, rel = H.hifde_gmres(F, torch.from_numpy(f).cuda(), tol=1e-12, maxit=50)
    u = u.cpu().numpy()
    ud = spla.spsolve(A.tocsc(), f)
    print("iterations", its.min(), its.max(), "relres", rel.max())
    assert np.all(rel <= 1e-12)
    err = np.linalg.norm(u - ud, axis=0) / np.linalg.norm(ud, axis=0)
    assert np.all(err <= 1e-9), err.max()
    F.free()
