"""Leading dimensions and in-place calls of hifde_solve, hifde_pcg and
hifde_gmres, through the C ABI: f and u with ld = N + pad, and u == f (the
header allows it for all three).  The results must equal the out-of-place ld = N call bit
for bit, and the padding rows must stay untouched.  Cases cover the 2D PCG
passes that walk strips of rows (ragged 48^2 grid, odd and even right-hand
side counts) and the 3D passes, in both precisions."""
import ctypes as C

import numpy as np
import pytest

from synth import workloads as W

from _helpers import gpu_factor, torch_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PAD = 37


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _padded(f, pad):
    """N x nrhs host array -> (nrhs, N + pad) device tensor (column-major
    N x nrhs with leading dimension N + pad); padding rows hold a marker."""
    N, nrhs = f.shape
    t = torch.full((nrhs, N + pad), 12345.0, dtype=torch.float64, device="cuda")
    t[:, :N] = torch.from_numpy(np.ascontiguousarray(f.T)).cuda()
    return t


def _call(F, which, nrhs, fp, ldf, up, ldu):
    import paper_1307_2895_amd as H
    lib = H.lib()
    if which == "solve":
        H.check(lib.hifde_solve(F._h, nrhs, C.c_void_p(fp), ldf, C.c_void_p(up), ldu, _stream()))
        return None
    its = (C.c_int * nrhs)()
    rel = (C.c_double * nrhs)()
    if which == "gmres":
        H.check(lib.hifde_gmres(F._h, nrhs, C.c_void_p(fp), ldf, C.c_void_p(up), ldu, 1e-12, 30,
                                200, its, rel, _stream()))
    else:
        H.check(lib.hifde_pcg(F._h, nrhs, C.c_void_p(fp), ldf, C.c_void_p(up), ldu, 1e-12, 200,
                              its, rel, _stream()))
    return list(its), list(rel)


@pytest.mark.parametrize("which", ["solve", "pcg", "gmres"])
@pytest.mark.parametrize("dim,n,m,nrhs,prec", [
    (2, 48, 3, 5, 0), (2, 48, 3, 34, 1), (2, 48, 3, 34, 0), (2, 48, 3, 5, 1),
    (3, 16, 4, 3, 1), (3, 16, 4, 4, 0),
])
def test_leading_dimension_and_in_place(which, dim, n, m, nrhs, prec):
    print(f"case {which} dim={dim} n={n} leaf={m} nrhs={nrhs} prec={prec}", flush=True)
    a = W.make_field(dim, n, "loguniform", 7)
    _, F = gpu_factor(dim, n, m, a, 1e-6, prec)
    N = n ** dim
    f = W.make_rhs(N, nrhs, 19)
    # reference: out of place, ld = N
    f0 = _padded(f, 0)
    u0 = torch.zeros_like(f0)
    r0 = _call(F, which, nrhs, f0.data_ptr(), N, u0.data_ptr(), N)
    # out of place with padded leading dimensions
    f1 = _padded(f, PAD)
    u1 = torch.full_like(f1, -777.0)
    r1 = _call(F, which, nrhs, f1.data_ptr(), N + PAD, u1.data_ptr(), N + PAD)
    # in place (u == f), padded
    f2 = _padded(f, PAD)
    r2 = _call(F, which, nrhs, f2.data_ptr(), N + PAD, f2.data_ptr(), N + PAD)
    torch.cuda.synchronize()
    assert torch.equal(u1[:, :N], u0)
    assert torch.equal(f2[:, :N], u0)
    assert bool((u1[:, N:] == -777.0).all()), "padding of u was written"
    assert bool((f1[:, N:] == 12345.0).all()) and bool((f1[:, :N] == f0).all()), "f was changed"
    assert bool((f2[:, N:] == 12345.0).all()), "padding of the in-place vector was written"
    if which != "solve":
        assert r0 == r1 == r2, (r0, r1, r2)
        assert max(r0[1]) <= 1.5e-12


@pytest.mark.parametrize("prec", [0, 2])
def test_gmres_columns_are_independent(prec):
    """A column's GMRES in a multi-column call (columns that converge at
    different steps, one of them zero) matches its single-column run: the
    same step count (one more or fewer where an estimate sits at the
    tolerance) and the solution to 1e-10."""
    import paper_1307_2895_amd as H
    n, m = 48, 3
    a = W.make_field(2, n, "loguniform", 7)
    b = np.full(n * n, -150.0)
    T = H.hifde_build_tree(2, n, m, 0)
    F = H.hifde_factor(T, torch_inputs(a), torch.from_numpy(b).cuda(), 1e-3, prec,
                       flags=H.HIFDE_INDEFINITE)
    f = W.make_rhs(n * n, 4, 23)
    f[:, 2] = 0.0
    f[:, 3] *= 1e-6
    U, its, rel = H.hifde_gmres(F, torch.from_numpy(f).cuda(), tol=1e-12, maxit=200)
    U = U.cpu().numpy()
    print("multi", its, rel)
    assert its[2] == 0 and np.all(U[:, 2] == 0.0)
    for c in (0, 1, 3):
        u, it1, r1 = H.hifde_gmres(F, torch.from_numpy(np.ascontiguousarray(f[:, c])).cuda(),
                                   tol=1e-12, maxit=200)
        u = u.cpu().numpy()
        print("column", c, it1, r1)
        assert abs(int(it1[0]) - int(its[c])) <= 1
        assert np.linalg.norm(U[:, c] - u) <= 1e-10 * np.linalg.norm(u)
    F.free()
