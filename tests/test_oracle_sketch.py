"""Pins of the randomized ID (Section 4.3's accelerated compression by a
Gaussian sampling matrix): the counter-based generator against its published
known-answer vectors and the normal law, and the ID of the sketch against
what the mathematics fixes."""
import numpy as np
import pytest
import scipy.stats as stats

from oracle import hifde as OH
from oracle import pcg as OP
from oracle import philox

# Known-answer vectors of Philox4x32-10 published with the generator
# (counter words, key words -> output words).
KAT = [
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff, 0xffffffff, 0xffffffff, 0xffffffff), (0xffffffff, 0xffffffff),
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(ctr, key, out):
    got = philox.philox4x32(*ctr, *key)
    assert tuple(int(x) for x in got) == out


def test_deviates_are_standard_normal():
    Z = philox.sketch_matrix(0, 7, 400, 500).ravel()
    assert abs(Z.mean()) < 5 / np.sqrt(Z.size)
    assert abs(Z.var() - 1.0) < 5 * np.sqrt(2.0 / Z.size)
    assert stats.kstest(Z, "norm").pvalue > 1e-3
    # different groups and levels draw different, uncorrelated matrices
    Z2 = philox.sketch_matrix(0, 8, 400, 500).ravel()
    Z3 = philox.sketch_matrix(1, 7, 400, 500).ravel()
    for other in (Z2, Z3):
        assert abs(np.corrcoef(Z, other)[0, 1]) < 5 / np.sqrt(Z.size)
    # a sub-block is the same draw (the counter is the element's position)
    assert np.array_equal(philox.sketch_matrix(3, 11, 5, 6),
                          philox.sketch_matrix(3, 11, 9, 10)[:5, :6])


def _decaying(m, n, rate, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (U * rate ** np.arange(n)) @ V.T


def test_id_is_invariant_under_orthogonal_sketches():
    """Column-pivoted QR of Q M has the R of M (up to row signs) for
    orthogonal Q, so the ID (skeletons, rank, T) is unchanged: the ID sees
    only the geometry of the columns, which a sketch approximately keeps."""
    M = _decaying(90, 40, 0.6, 0)
    Q, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((90, 90)))
    a = OH.interp_decomp(M, 1e-6)
    b = OH.interp_decomp(Q @ M, 1e-6)
    assert a.k == b.k and np.array_equal(a.perm, b.perm)
    np.testing.assert_allclose(a.T, b.T, rtol=1e-8, atol=1e-10)


def test_sketch_recovers_exact_low_rank():
    """rank(M) = 12 < 30 sampled rows: with probability one the sketch keeps
    the column space, the ID has rank 12 and reproduces M to rounding."""
    rng = np.random.default_rng(2)
    M = rng.standard_normal((150, 12)) @ rng.standard_normal((12, 30))
    Phi = philox.sketch_matrix(2, 5, 30, 150)
    idr = OH.interp_decomp(Phi @ M, 1e-10)
    assert idr.k == 12
    sk, rd = idr.perm[:12], idr.perm[12:]
    err = np.linalg.norm(M[:, rd] - M[:, sk] @ idr.T) / np.linalg.norm(M)
    assert err < 1e-10


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_sketched_id_error_tracks_the_deterministic_one(seed):
    """Singular values 0.7^j, eps = 1e-6: the ID of the (|c| + 16) x |c|
    sketch of the 5|c| x |c| block keeps the deterministic rank within 3 and
    its error ||M - M_S T||_2 within 10 eps ||M||_2 sqrt(|c|)."""
    n = 48
    M = _decaying(5 * n, n, 0.7, seed)
    det = OH.interp_decomp(M, 1e-6)
    rows = philox.sketch_rows(n, 5 * n)
    assert rows == n + 16
    Phi = philox.sketch_matrix(1, 100 + seed, rows, 5 * n)
    rnd = OH.interp_decomp(Phi @ M, 1e-6)
    assert abs(rnd.k - det.k) <= 3, (rnd.k, det.k)
    sk, rd = rnd.perm[:rnd.k], rnd.perm[rnd.k:]
    err = np.linalg.norm(M[:, rd] - M[:, sk] @ rnd.T, 2) / np.linalg.norm(M, 2)
    assert err <= 10 * 1e-6 * np.sqrt(n), err


@pytest.mark.parametrize("dim,n,m", [(2, 64, 8), (3, 16, 4)])
def test_sketched_factorization_preconditions_as_well(dim, n, m):
    """The sketched factorization has the same cells and groups, an
    approximation error within 10x of the deterministic one (about 1.3x in
    2D and 3x in 3D here; without the 16 extra rows 30x), and PCG converges
    in about as many iterations."""
    from synth import workloads as W
    a = W.make_field(dim, n, "bernoulli_contrast", 2)
    f = W.make_rhs(n ** dim, 1, 3)[:, 0]
    Fd = OH.factor(dim, n, m, a, eps=1e-6)
    Fs = OH.factor(dim, n, m, a, eps=1e-6, sketch=True)
    for ld, ls in zip(Fd.levels, Fs.levels):
        assert [c.cid for c in ld.cells] == [c.cid for c in ls.cells]
        assert [g.gid for g in ld.groups] == [g.gid for g in ls.groups]
        # the first level's groups are formed before any skeleton choice
        break
    rng = np.random.default_rng(6)
    x = rng.standard_normal(n ** dim)
    nA = np.linalg.norm(Fd.A @ x)
    ed = np.linalg.norm(Fd.A @ x - OH.apply(Fd, x)) / nA
    es = np.linalg.norm(Fs.A @ x - OH.apply(Fs, x)) / nA
    print("e_a deterministic", ed, "sketched", es)
    assert es <= 10 * max(ed, 1e-12)
    _, itd, _ = OP.pcg(Fd.A, f, lambda r: OH.solve(Fd, r), 1e-12, 100)
    _, its, rr = OP.pcg(Fs.A, f, lambda r: OH.solve(Fs, r), 1e-12, 100)
    print("pcg iterations", itd, its)
    assert rr <= 1e-11 and its <= itd + 3
