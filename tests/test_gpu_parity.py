"""GPU parity: the HIP path against the FP64 oracle on the same seeded inputs.

Bars (stated per test): index sets bit-exact in FP64; relative residual of
one F^-1 application within 2x of the oracle's at the same eps; PCG-refined
solutions within 1e-10 of the oracle (as ||A (u_gpu - u_ora)|| / ||f||).
"""
import numpy as np
import pytest

from oracle import hifde as OH
from oracle import pcg as OP
from synth import workloads as W

from _helpers import compare_sets, compare_structure, gpu_factor, oracle_factor, rel_residual

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solve(F, f):
    import paper_1307_2895_amd as H
    u = H.hifde_solve(F, torch.from_numpy(np.ascontiguousarray(f)).cuda())
    return u.cpu().numpy()


CASES_FP64 = [
    # dim, n, leaf, eps, field, seed
    (2, 64, 8, 1e-6, "const", None),            # the 2D Laplacian workload, N=4096
    (2, 64, 8, 1e-6, "bernoulli_contrast", 2),   # high contrast at the small size
    (2, 48, 3, 1e-6, "loguniform", 7),           # ragged: leaf 3, L=4
    (2, 32, 4, 0.0, "loguniform", 5),            # eps = 0: exact multifrontal
    (3, 16, 4, 1e-6, "const", None),
    (3, 16, 2, 1e-3, "lognormal_grf", 4),
    # natural sizes: the one-launch level-0 upward sweep, the whole-front and
    # fused-interpolation sweeps (2D, 4096 level-0 cells), the wide ID
    # (groups of 128 and more unknowns) and the wide extend-add (fronts of
    # 512 and more) all run at their default launch choices (3D)
    (2, 512, 8, 1e-6, "bernoulli_contrast", 2),
    (3, 32, 4, 1e-6, "const", None),
]


@pytest.mark.parametrize("dim,n,m,eps,field,seed", CASES_FP64)
def test_fp64_parity(dim, n, m, eps, field, seed):
    print(f"case dim={dim} n={n} leaf={m} eps={eps} field={field}", flush=True)
    a = W.make_field(dim, n, field, seed)
    OF = oracle_factor(dim, n, m, a, eps)
    T, F = gpu_factor(dim, n, m, a, eps, 0)
    cm, gm, sm, first = compare_sets(OF, F)
    assert cm == 0 and gm == 0, (cm, gm)
    assert sm == 0, f"{sm} skeleton sets differ (first at level {first})"
    N = n ** dim
    f = W.make_rhs(N, 3, 11)
    u = _solve(F, f)
    ur = OH.solve(OF, f)
    rg = rel_residual(OF.A, u, f)
    ro = rel_residual(OF.A, ur, f)
    print("residual gpu", rg, "oracle", ro)
    if eps == 0.0:
        assert np.all(rg < 1e-12)
    else:
        assert np.all(rg <= 2.0 * ro)
    # same factorization: F^-1 f agrees with the oracle's to the accuracy of
    # the arithmetic (both FP64, identical skeletons)
    assert np.max(np.abs(u - ur)) <= 1e-8 * np.max(np.abs(ur))


def test_fp64_pcg_matches_oracle():
    import paper_1307_2895_amd as H
    w = W.workload("laplace2d_n64")
    a = W.make_coefficients(w)
    OF = oracle_factor(w.dim, w.n, w.leaf, a, w.eps)
    T, F = gpu_factor(w.dim, w.n, w.leaf, a, w.eps, 0)
    f = W.make_rhs(w.N, 2, w.seed_f)
    ug, its, rel = H.hifde_pcg(F, torch.from_numpy(f).cuda(), tol=1e-12, maxit=100)
    ug = ug.cpu().numpy()
    uo, ito, relo = OP.pcg_multi(OF.A, f, lambda r: OH.solve(OF, r), 1e-12, 100)
    assert np.all(rel <= 1e-12 * 1.5), rel
    d = np.linalg.norm(OF.A @ (ug - uo), axis=0) / np.linalg.norm(f, axis=0)
    assert np.all(d <= 1e-10), d
    print("iters gpu", its, "oracle", ito)
    assert np.all(np.abs(its - ito) <= 1)


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("dim,n,m,eps,field,seed", [
    (2, 64, 8, 1e-6, "const", None),
    (2, 64, 8, 1e-6, "bernoulli_contrast", 2),
    (3, 16, 4, 1e-6, "const", None),
])
def test_mixed_pcg_converges(dim, n, m, eps, field, seed, prec):
    import paper_1307_2895_amd as H
    a = W.make_field(dim, n, field, seed)
    OF = oracle_factor(dim, n, m, a, eps)
    T, F = gpu_factor(dim, n, m, a, eps, prec)
    # the structural sets of level 0 and level 1/2 do not depend on any
    # skeleton choice: bit-exact in mixed precision too
    cm, gm = compare_structure(OF, F, levels=1)
    assert cm == 0 and gm == 0, (cm, gm)
    N = n ** dim
    f = W.make_rhs(N, 4, 13)
    ug, its, rel = H.hifde_pcg(F, torch.from_numpy(f).cuda(), tol=1e-12, maxit=200)
    ug = ug.cpu().numpy()
    assert np.all(rel <= 1.5e-12), rel
    uo, ito, _ = OP.pcg_multi(OF.A, f, lambda r: OH.solve(OF, r), 1e-12, 200)
    d = np.linalg.norm(OF.A @ (ug - uo), axis=0) / np.linalg.norm(f, axis=0)
    assert np.all(d <= 1e-10), d
    print("mixed iters", its, "oracle fp64 iters", ito)


# Right-hand-side counts that change the PCG passes' 2D strips: 5 columns run
# one column per lane (strips 51 unknowns wide, one per row of 48), 34 run
# pairs of columns (strips 15 wide: four per row, the last one ragged).
@pytest.mark.parametrize("mixed", [0, 1, 2])
@pytest.mark.parametrize("nrhs", [5, 34])
def test_pcg_ragged_strips_match_oracle(mixed, nrhs):
    import paper_1307_2895_amd as H
    dim, n, m, eps = 2, 48, 3, 1e-6
    print(f"case n={n} leaf={m} nrhs={nrhs} mixed={mixed}", flush=True)
    a = W.make_field(dim, n, "loguniform", 7)
    OF = oracle_factor(dim, n, m, a, eps)
    T, F = gpu_factor(dim, n, m, a, eps, mixed)
    f = W.make_rhs(n ** dim, nrhs, 17)
    ug, its, rel = H.hifde_pcg(F, torch.from_numpy(f).cuda(), tol=1e-12, maxit=200)
    ug = ug.cpu().numpy()
    assert np.all(rel <= 1.5e-12), rel
    uo, ito, _ = OP.pcg_multi(OF.A, f, lambda r: OH.solve(OF, r), 1e-12, 200)
    d = np.linalg.norm(OF.A @ (ug - uo), axis=0) / np.linalg.norm(f, axis=0)
    assert np.all(d <= 1e-10), d
    print("iters gpu", its, "oracle", ito)
    if not mixed:
        assert np.all(np.abs(its - ito) <= 1)


def test_fp64_pcg_to_stagnation_matches_oracle():
    """Second check of the PCG solutions (Laplacian 64^2, kappa ~ 1.7e3 < 1e4):
    both sides iterate to 1e-14 or to stagnation (30 iterations) and the
    solutions agree to a relative 2-norm difference of 1e-10."""
    import paper_1307_2895_amd as H
    w = W.workload("laplace2d_n64")
    a = W.make_coefficients(w)
    OF = oracle_factor(w.dim, w.n, w.leaf, a, w.eps)
    T, F = gpu_factor(w.dim, w.n, w.leaf, a, w.eps, 0)
    f = W.make_rhs(w.N, 2, w.seed_f)
    ug, its, rel = H.hifde_pcg(F, torch.from_numpy(f).cuda(), tol=1e-14, maxit=30,
                               raise_on_noconv=False)
    ug = ug.cpu().numpy()
    uo, ito, relo = OP.pcg_multi(OF.A, f, lambda r: OH.solve(OF, r), 1e-14, 30)
    d = np.linalg.norm(ug - uo, axis=0) / np.linalg.norm(uo, axis=0)
    print("iters gpu", its, "oracle", ito, "relres gpu", rel, "oracle", relo, "rel diff", d)
    assert np.all(rel <= 1e-13) and np.all(relo <= 1e-13)
    assert np.all(d <= 1e-10), d
