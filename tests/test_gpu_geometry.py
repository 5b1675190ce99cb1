"""Grids beyond the uniform tree on the GPU: sides that leaf * 2^L does not
divide (the last box along each axis is short, as on the paper's
n = 2^k - 1 grids) and zero-flux (Neumann) sides from zero boundary-link
coefficients.  Same bars as the uniform parity tests: FP64 index sets bit
for bit against the oracle, F^-1 f within 1e-8, the one-application
residual within 2x; the mixed precision converges in PCG to the oracle's
solution."""
import numpy as np
import pytest

from oracle import hifde as OH
from oracle import pcg as OP
from synth import workloads as W

from _helpers import compare_sets, rel_residual, torch_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _neumann(a, dim, sides):
    """Zero the boundary links of the given sides: (axis, 0) is x_axis = 0,
    (axis, 1) is x_axis = n - 1."""
    out = [x.copy() for x in a]
    for axis, hi in sides:
        pos = dim - 1 - axis                 # C-order position of the axis
        sl = [slice(None)] * dim
        sl[pos] = -1 if hi else 0
        out[axis][tuple(sl)] = 0.0
    return out


CASES = [
    # dim, n, leaf, eps, field, seed, zero-flux sides
    (2, 60, 8, 1e-6, "bernoulli_contrast", 2, []),
    (2, 57, 8, 1e-3, "loguniform", 7, []),            # last leaf box one wide
    (3, 30, 4, 1e-6, "const", None, []),
    (2, 511, 8, 1e-6, "bernoulli_contrast", 2, []),    # the paper's 2^k - 1 form
    (2, 64, 8, 1e-6, "bernoulli_contrast", 2, [(0, 0), (1, 1)]),
    (3, 16, 4, 1e-6, "const", None, [(2, 0)]),
    (2, 60, 8, 1e-6, "loguniform", 3, [(0, 0), (0, 1), (1, 0)]),
]


def _case(dim, n, m, field, seed, sides):
    return _neumann(W.make_field(dim, n, field, seed), dim, sides)


@pytest.mark.parametrize("dim,n,m,eps,field,seed,sides", CASES)
def test_geometry_fp64_parity(dim, n, m, eps, field, seed, sides):
    import paper_1307_2895_amd as H
    print(f"case geometry dim={dim} n={n} leaf={m} eps={eps} sides={sides}", flush=True)
    a = _case(dim, n, m, field, seed, sides)
    OF = OH.factor(dim, n, m, a, eps=eps)
    T = H.hifde_build_tree(dim, n, m, 0)
    F = H.hifde_factor(T, torch_inputs(a), None, eps, H.HIFDE_FP64)
    assert H.hifde_stats(F)["levels"] == OF.L
    cm, gm, sm, first = compare_sets(OF, F)
    assert cm == 0 and gm == 0, (cm, gm)
    assert sm == 0, f"{sm} skeleton sets differ (first at level {first})"
    f = W.make_rhs(n ** dim, 3, 11)
    u = H.hifde_solve(F, torch.from_numpy(f).cuda()).cpu().numpy()
    ur = OH.solve(OF, f)
    rg, ro = rel_residual(OF.A, u, f), rel_residual(OF.A, ur, f)
    diff = np.linalg.norm(u - ur) / np.linalg.norm(ur)
    print("residual gpu", rg, "oracle", ro, "F^-1 f difference", diff)
    assert diff <= 1e-8
    assert np.all(rg <= 2 * ro + 1e-14)
    F.free()


@pytest.mark.parametrize("dim,n,m,field,seed,sides", [
    (2, 60, 8, "bernoulli_contrast", 2, []),
    (2, 64, 8, "bernoulli_contrast", 2, [(0, 0), (1, 1)]),
    (3, 30, 4, "const", None, [(2, 0)]),
])
def test_geometry_mixed_pcg(dim, n, m, field, seed, sides):
    import paper_1307_2895_amd as H
    print(f"case geometry mixed dim={dim} n={n} sides={sides}", flush=True)
    a = _case(dim, n, m, field, seed, sides)
    OF = OH.factor(dim, n, m, a, eps=1e-6)
    f = W.make_rhs(n ** dim, 2, 12)
    uo, _, _ = OP.pcg_multi(OF.A, f, lambda r: OH.solve(OF, r), 1e-12, 100)
    T = H.hifde_build_tree(dim, n, m, 0)
    F = H.hifde_factor(T, torch_inputs(a), None, 1e-6, H.HIFDE_MIXED_ELIM64)
    u, its, rel = H.hifde_pcg(F, torch.from_numpy(f).cuda(), tol=1e-12, maxit=100)
    u = u.cpu().numpy()
    print("iterations", its, "relres", rel)
    assert np.all(rel <= 1.5e-12)
    err = np.linalg.norm(OF.A @ (u - uo), axis=0) / np.linalg.norm(f, axis=0)
    assert np.all(err <= 1e-10), err
    F.free()


def test_negative_boundary_link_rejected():
    import paper_1307_2895_amd as H
    n, m = 32, 4
    a = W.make_field(2, n, "const", None)
    a[0][:, 0] = -1.0
    T = H.hifde_build_tree(2, n, m, 0)
    with pytest.raises(H.HifdeError) as ei:
        H.hifde_factor(T, torch_inputs(a), None, 1e-6, H.HIFDE_FP64)
    assert ei.value.code == H.HIFDE_EINVAL
    a[0][:, 0] = 0.0
    F = H.hifde_factor(T, torch_inputs(a), None, 1e-6, H.HIFDE_FP64)
    F.free()
