"""Pins of the oracle's discretization against facts that do not depend on
its code: the DST-I eigendecomposition of the constant-coefficient Laplacian
and the energy identity of the staggered five/seven-point stencil."""
import numpy as np
import pytest
import scipy.fft

from oracle import problem
from synth import workloads as W


def _dst_solve(dim, n, f):
    """Exact A^-1 f for a = 1, b = 0: A = S diag(lambda) S with the orthonormal
    DST-I matrix S and lambda = h^-2 sum_k 4 sin^2(j_k pi h / 2)."""
    h = 1.0 / (n + 1)
    j = np.arange(1, n + 1)
    lam1 = 4.0 * np.sin(j * np.pi * h / 2.0) ** 2 / h ** 2
    grids = np.meshgrid(*([lam1] * dim), indexing="ij")
    lam = sum(grids)
    F = f.reshape((n,) * dim)
    G = scipy.fft.dstn(F, type=1, norm="ortho")
    return scipy.fft.idstn(G / lam, type=1, norm="ortho").ravel()


@pytest.mark.parametrize("dim,n", [(2, 12), (2, 31), (3, 7)])
def test_constant_coefficient_matches_dst(dim, n):
    a = W.make_field(dim, n, "const", None)
    A = problem.assemble(dim, n, a)
    f = np.random.default_rng(0).standard_normal(n ** dim)
    u = _dst_solve(dim, n, f)
    assert np.linalg.norm(A @ u - f) <= 1e-12 * np.linalg.norm(f)


@pytest.mark.parametrize("dim,n", [(2, 5), (3, 4)])
def test_energy_identity(dim, n):
    """u^T A u = h^-2 sum_links a_link (u_i - u_j)^2 + sum_i b_i u_i^2, with
    u = 0 outside the grid: fixes every entry of the symmetric A."""
    rng = np.random.default_rng(1)
    a = W.make_field(dim, n, "loguniform", 3)
    b = rng.uniform(0.0, 2.0, n ** dim)
    A = problem.assemble(dim, n, a, b)
    h2inv = (n + 1.0) ** 2
    for _ in range(3):
        u = rng.standard_normal(n ** dim)
        U = u.reshape((n,) * dim)            # axes x_{d-1}, ..., x0
        energy = float(np.sum(b * u * u))
        for k in range(dim):
            ax = dim - 1 - k                 # numpy axis of coordinate x_k
            pad = [(0, 0)] * dim
            pad[ax] = (1, 1)
            Up = np.pad(U, pad)              # zeros on the boundary layers
            diff = np.diff(Up, axis=ax)      # n+1 links along axis k
            energy += h2inv * float(np.sum(a[k] * diff * diff))
        assert abs(u @ (A @ u) - energy) <= 1e-12 * abs(energy)
    assert abs(A - A.T).max() == 0.0


def test_coefficient_layout():
    """a[k] has n+1 entries along axis k and n along the others."""
    for dim in (2, 3):
        for k in range(dim):
            s = W.coeff_shape(dim, 5, k)
            assert s[dim - 1 - k] == 6 and sum(s) == 5 * dim + 1


def test_zero_boundary_links_give_neumann_sides():
    """A zero coefficient on the boundary links of the x0 = 0 side removes
    their Dirichlet term (a zero-flux side, first order): along x0 the
    matrix is h^-2 tridiag(-1, 2, -1) with first entry 1, whose eigenvalues
    are 2 - 2 cos((2j - 1) pi / (2n + 1)); A is the Kronecker sum with the
    Dirichlet axis, 2 - 2 cos(j pi / (n + 1))."""
    n = 12
    a = [np.ones((n, n + 1)), np.ones((n + 1, n))]
    a[0][:, 0] = 0.0                     # links 0 along axis 0 (x0 = 0 side)
    A = problem.assemble(2, n, a)
    j = np.arange(1, n + 1)
    lam_n = 2 - 2 * np.cos((2 * j - 1) * np.pi / (2 * n + 1))
    lam_d = 2 - 2 * np.cos(j * np.pi / (n + 1))
    want = np.sort((lam_n[:, None] + lam_d[None, :]).ravel()) * (n + 1) ** 2
    got = np.linalg.eigvalsh(A.toarray())
    np.testing.assert_allclose(got, want, rtol=1e-10)
