"""Leading dimensions and in-place calls of hifde_solve and hifde_pcg,
through the C ABI: f and u with ld = N + pad, and u == f (the header allows
it for both calls).  The results must equal the out-of-place ld = N call bit
for bit, and the padding rows must stay untouched.  Cases cover the 2D PCG
passes that walk strips of rows (ragged 48^2 grid, odd and even right-hand
side counts) and the 3D passes, in both precisions."""
import ctypes as C

import numpy as np
import pytest

from synth import workloads as W

from _helpers import gpu_factor

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
    H.check(lib.hifde_pcg(F._h, nrhs, C.c_void_p(fp), ldf, C.c_void_p(up), ldu, 1e-12, 200,
                          its, rel, _stream()))
    return list(its), list(rel)


@pytest.mark.parametrize("which", ["solve", "pcg"])
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
    if which == "pcg":
        assert r0 == r1 == r2, (r0, r1, r2)
        assert max(r0[1]) <= 1.5e-12
