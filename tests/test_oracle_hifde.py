"""Pins of the oracle's HIF-DE against the paper's lemmas, exact special
cases, library routines and invariants."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import errest as OE
from oracle import hifde as OH
from oracle import problem
from synth import workloads as W

from test_oracle_problem import _dst_solve

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _spd(n, rng, cond=1e3):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T


# ---------------------------------------------------------------- Lemma 2.1
def test_lemma_2_1_block_diagonalizes():
    rng = np.random.default_rng(0)
    p, q, r = 7, 5, 6
    A = _spd(p + q + r, rng)
    ip, iq, ir = np.arange(p), np.arange(p, p + q), np.arange(p + q, p + q + r)
    A[np.ix_(ip, ir)] = 0.0
    A[np.ix_(ir, ip)] = 0.0
    A += (p + q + r) * 10 * np.eye(p + q + r)   # keep it SPD after zeroing
    L, D, Wm, upd = OH.sparse_elimination(A[np.ix_(ip, ip)], A[np.ix_(iq, ip)])
    S = np.eye(p + q + r)
    Linv_T = np.linalg.inv(L).T
    S[np.ix_(ip, ip)] = Linv_T
    S[np.ix_(ip, iq)] = -Linv_T @ Wm
    B = S.T @ A @ S
    assert np.allclose(B[np.ix_(ip, ip)], np.diag(D), atol=1e-12 * np.abs(A).max())
    assert np.abs(B[np.ix_(ip, iq)]).max() <= 1e-12 * np.abs(A).max()
    assert np.abs(B[np.ix_(ip, ir)]).max() <= 1e-12 * np.abs(A).max()
    schur = A[np.ix_(iq, iq)] - A[np.ix_(iq, ip)] @ np.linalg.solve(A[np.ix_(ip, ip)], A[np.ix_(ip, iq)])
    assert np.allclose(B[np.ix_(iq, iq)], schur, rtol=1e-12, atol=1e-12 * np.abs(A).max())
    assert np.allclose(A[np.ix_(iq, iq)] + upd, schur, atol=1e-12 * np.abs(A).max())
    assert np.array_equal(B[np.ix_(ir, ir)], A[np.ix_(ir, ir)])


def test_ldl_reconstructs():
    rng = np.random.default_rng(1)
    A = _spd(9, rng)
    L, D = OH.ldl_spd(A)
    assert np.allclose(np.diag(L), 1.0) and np.allclose(np.triu(L, 1), 0.0)
    assert np.allclose((L * D) @ L.T, A, atol=1e-12 * np.abs(A).max())
    with pytest.raises(OH.NotSPD):
        OH.ldl_spd(-A)


# ---------------------------------------------------------------- ID (Section 2.2)
@pytest.mark.parametrize("m,n", [(30, 12), (12, 30), (50, 50)])
def test_id_pivots_match_lapack(m, n):
    """On generic matrices (no ties) the pivots and |R_jj| agree with
    LAPACK's column-pivoted QR (dgeqp3)."""
    rng = np.random.default_rng(m * 100 + n)
    M = rng.standard_normal((m, n))
    res = OH.interp_decomp(M, 1e-15)
    Q, R, P = sla.qr(M, pivoting=True, mode="economic")
    k = res.k
    assert k == min(m, n)
    assert np.array_equal(res.perm[:k], P[:k])
    assert np.allclose(res.rdiag, np.abs(np.diag(R))[:k], rtol=1e-12)


def test_id_exact_low_rank():
    rng = np.random.default_rng(2)
    m, n, k0 = 40, 25, 7
    M = rng.standard_normal((m, k0)) @ rng.standard_normal((k0, n))
    res = OH.interp_decomp(M, 1e-10)
    assert res.k == k0
    sk, rd = res.perm[:k0], res.perm[k0:]
    E = M[:, rd] - M[:, sk] @ res.T
    assert np.linalg.norm(E) <= 1e-12 * np.linalg.norm(M)


def test_id_tolerance_and_bounds():
    """Adaptive rank: ||E|| <~ eps ||A|| and the typical bound
    ||T|| <= sqrt(4 k (n - k)) (Section 2.2), on smooth kernel blocks."""
    x = np.linspace(0, 1, 60)
    y = np.linspace(2, 3, 30)
    M = 1.0 / np.abs(x[:, None] - y[None, :])
    for eps in (1e-4, 1e-8):
        res = OH.interp_decomp(M, eps)
        k, n = res.k, M.shape[1]
        E = M[:, res.perm[k:]] - M[:, res.perm[:k]] @ res.T
        assert 0 < k < n
        assert np.linalg.norm(E, 2) <= 10 * eps * np.linalg.norm(M, 2)
        assert np.linalg.norm(res.T, 2) <= np.sqrt(4 * k * (n - k))


def test_id_ties_go_to_lowest_position():
    M = np.array([[1.0, 1.0, 0.5], [1.0, 1.0, 0.2]])
    M = np.hstack([M[:, [2]], M[:, :2]])       # equal-norm columns at positions 1, 2
    res = OH.interp_decomp(M, 1e-12)
    assert res.perm[0] == 1


# ---------------------------------------------------------------- Lemma 2.4
def test_lemma_2_4_skeletonization():
    """With an exactly low-rank A_qp, S_r^T Q^T A Q S_r is block diagonal and
    the skeleton block is B_ss (the truncation drops nothing)."""
    rng = np.random.default_rng(3)
    p, q, k0 = 9, 14, 4
    Aqp = rng.standard_normal((q, k0)) @ rng.standard_normal((k0, p))
    A = np.zeros((p + q, p + q))
    A[:p, :p] = _spd(p, rng)
    A[p:, p:] = _spd(q, rng)
    A[p:, :p] = Aqp
    A[:p, p:] = Aqp.T
    A += 100 * np.eye(p + q)
    res = OH.interp_decomp(Aqp, 1e-12)
    assert res.k == k0
    sk = np.sort(res.perm[:k0])
    rd = np.sort(res.perm[k0:])
    T = res.T[np.argsort(res.perm[:k0])][:, np.argsort(res.perm[k0:])]
    Lr, Dr, Wr, Bss = OH.skeletonize_block(A[np.ix_(rd, rd)], A[np.ix_(sk, rd)], A[np.ix_(sk, sk)], T)
    # explicit operators on the ordering (r, s, q)
    order = np.concatenate([rd, sk, p + np.arange(q)])
    Ao = A[np.ix_(order, order)]
    r, k = rd.size, sk.size
    Q = np.eye(p + q)
    Q[r:r + k, :r] = -T
    S = np.eye(p + q)
    LrinvT = np.linalg.inv(Lr).T
    S[:r, :r] = LrinvT
    S[:r, r:r + k] = -LrinvT @ Wr
    Z = S.T @ Q.T @ Ao @ Q @ S
    scale = np.abs(A).max()
    assert np.allclose(Z[:r, :r], np.diag(Dr), atol=1e-11 * scale)
    assert np.abs(Z[:r, r:]).max() <= 1e-11 * scale
    assert np.allclose(Z[r:r + k, r:r + k], Bss, atol=1e-11 * scale)
    assert np.allclose(Z[r + k:, r:r + k], Ao[r + k:, r:r + k], atol=1e-11 * scale)


# ---------------------------------------------------------------- Algorithm 4.1
@pytest.mark.parametrize("dim,n,m", [(2, 32, 4), (2, 48, 3), (3, 8, 2), (3, 12, 3)])
def test_eps0_is_exact_dst(dim, n, m):
    """eps = 0 is the multifrontal method: F = A, checked against the DST-I
    closed-form solve (a = 1)."""
    a = W.make_field(dim, n, "const", None)
    F = OH.factor(dim, n, m, a, eps=0.0)
    f = np.random.default_rng(4).standard_normal(n ** dim)
    u = OH.solve(F, f)
    ue = _dst_solve(dim, n, f)
    assert np.linalg.norm(u - ue) <= 1e-12 * np.linalg.norm(ue)


@pytest.mark.parametrize("dim,n,m,field", [(2, 32, 4, "bernoulli_contrast"), (2, 24, 3, "loguniform"),
                                           (3, 12, 3, "lognormal_grf")])
def test_eps0_is_exact_sparse_direct(dim, n, m, field):
    a = W.make_field(dim, n, field, 5)
    F = OH.factor(dim, n, m, a, eps=0.0)
    f = np.random.default_rng(5).standard_normal(n ** dim)
    u = OH.solve(F, f)
    ue = spla.spsolve(F.A.tocsc(), f)
    assert np.linalg.norm(u - ue) <= 1e-11 * np.linalg.norm(ue)


def _dense_F(F):
    return OH.apply(F, np.eye(F.N))


@pytest.mark.parametrize("dim,n,m,eps,field", [(2, 16, 4, 1e-6, "const"), (2, 16, 2, 1e-3, "loguniform"),
                                               (3, 8, 2, 1e-6, "const"), (2, 16, 4, 1e-2, "bernoulli_contrast")])
def test_weyl_and_spd(dim, n, m, eps, field):
    """Theorem 4.1 and its corollary: F is symmetric; when eps kappa(A) < 1 it
    is SPD, and every eigenvalue is within a relative e_a kappa(A) of A's."""
    a = W.make_field(dim, n, field, 6)
    F = OH.factor(dim, n, m, a, eps=eps)
    A = F.A.toarray()
    Fd = _dense_F(F)
    assert np.abs(Fd - Fd.T).max() <= 1e-12 * np.abs(A).max()
    Fd = 0.5 * (Fd + Fd.T)
    la = np.linalg.eigvalsh(A)
    lf = np.linalg.eigvalsh(Fd)
    ea = np.linalg.norm(A - Fd, 2) / np.linalg.norm(A, 2)
    kappa = la[-1] / la[0]
    assert np.all(np.abs(la - lf) / la <= ea * kappa * (1 + 1e-8) + 1e-13)
    if ea * kappa < 1:
        assert lf.min() > 0
    # F^-1 applied in factored form is the inverse of F applied in factored form
    Finv = OH.solve(F, np.eye(F.N))
    assert np.abs(Finv @ Fd - np.eye(F.N)).max() <= 1e-8


@pytest.mark.parametrize("dim,n,m,eps", [(2, 64, 8, 1e-6), (2, 64, 8, 1e-9), (3, 16, 4, 1e-6), (3, 16, 4, 1e-3)])
def test_accuracy_order_eps(dim, n, m, eps):
    """e_a = O(eps) (Tables 2, 8): between 0.05 eps and 100 eps."""
    a = W.make_field(dim, n, "const", None)
    F = OH.factor(dim, n, m, a, eps=eps)
    ea = OE.e_a(F.A, lambda v: OH.apply(F, v))
    assert 0.05 * eps <= ea <= 100 * eps


def test_power_iteration_matches_dense():
    a = W.make_field(2, 16, "loguniform", 8)
    F = OH.factor(2, 16, 4, a, eps=1e-4)
    A = F.A.toarray()
    Fd = _dense_F(F)
    Finv = OH.solve(F, np.eye(F.N))
    es_dense = np.linalg.norm(np.eye(F.N) - A @ Finv, 2)
    ea_dense = np.linalg.norm(A - Fd, 2) / np.linalg.norm(A, 2)
    es = OE.e_s(F.A, lambda v: OH.solve(F, v))
    ea = OE.e_a(F.A, lambda v: OH.apply(F, v))
    assert abs(es - es_dense) <= 5e-2 * es_dense
    assert abs(ea - ea_dense) <= 5e-2 * ea_dense


def test_inverse_symmetric():
    a = W.make_field(2, 32, "bernoulli_contrast", 2)
    F = OH.factor(2, 32, 4, a, eps=1e-6)
    rng = np.random.default_rng(7)
    x, y = rng.standard_normal(F.N), rng.standard_normal(F.N)
    lhs, rhs = x @ OH.solve(F, y), y @ OH.solve(F, x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_paper_magnitudes():
    """Sanity bands around the paper's printed 2D Laplacian numbers
    (Tables 1-2, eps = 1e-6: |s_L| 52-57, e_a ~ 1e-5, n_i <= 15): our grids
    are smaller, so only the orders of magnitude must agree."""
    with open(os.path.join(GOLDEN, "paper_tables.json")) as fh:
        gold = json.load(fh)
    row = gold["table1_2_hifde2_eps1e-6"][0]
    a = W.make_field(2, 256, "const", None)
    F = OH.factor(2, 256, 16, a, eps=1e-6)
    assert 0.5 * row["sL"] <= F.top_size <= 1.5 * row["sL"]
    ea = OE.e_a(F.A, lambda v: OH.apply(F, v))
    assert row["e_a"] / 100 <= ea <= row["e_a"] * 10


# ---------------------------------------------------------------- flop count
def _one_level_closed_form(dim, m):
    """Sizes of the one-level tree n = 2m (Section 3.1's geometry): the
    2^dim cells have extents e_j in {m-1, m} (the last box per axis holds
    one more row), interiors p = prod e_j and fronts q = sum_k prod_{j!=k}
    e_j (the separator faces they touch; corner lines are not stencil
    neighbours of an interior).  Each separator face on plane k with
    extents e_j (j != k) has |c| = prod e_j and, after the cells are
    eliminated, |c^N| = 2m sum_j prod_{i!=j} e_i: the other faces of its two
    cells ((2m-1) e per crossing axis) plus the corner-line unknowns next
    to it (one e per crossing axis)."""
    import itertools
    ext = (m - 1, m)
    cells = []
    for idx in itertools.product((0, 1), repeat=dim):
        e = [ext[i] for i in idx]
        p = int(np.prod(e))
        q = sum(int(np.prod([e[j] for j in range(dim) if j != k])) for k in range(dim))
        cells.append((p, q))
    groups = []
    for k in range(dim):
        others = [j for j in range(dim) if j != k]
        for idx in itertools.product((0, 1), repeat=dim - 1):
            e = [ext[i] for i in idx]
            c = int(np.prod(e))
            cN = 2 * m * sum(int(np.prod([e[i] for i in range(len(e)) if i != j]))
                             for j in range(len(e)))
            groups.append((c, cN))
    return cells, groups


@pytest.mark.parametrize("dim,m,eps,field", [(2, 8, 0.0, "const"), (2, 8, 1e-6, "const"),
                                             (2, 7, 1e-4, "loguniform"), (3, 4, 0.0, "const"),
                                             (3, 4, 1e-6, "loguniform")])
def test_factor_flops_closed_form_one_level(dim, m, eps, field):
    """factor_flops on n = 2m (one level) equals the dense-block count
    written from the closed-form sizes: cells p^3/3 + p^2 q + p q^2 (Lemma
    2.1), skeletonized groups 2|c^N||c|k + r^3/3 + 5kr^2 + 4k^2r (Section
    2.2 and Lemma 2.4) and the top |s_L|^3/3, |s_L| = N - sum p - sum r.
    The group ranks k are the oracle's (the count takes them as given)."""
    n = 2 * m
    a = W.make_field(dim, n, field, 3)
    F = OH.factor(dim, n, m, a, eps=eps)
    cells, groups = _one_level_closed_form(dim, m)
    assert F.L == 1
    got_cells = sorted((c.p.size, c.q.size) for c in F.levels[0].cells)
    assert got_cells == sorted(cells)
    got_groups = sorted((g.c.size, g.cN.size) for g in F.levels[0].groups)
    assert got_groups == sorted(groups)
    fl = sum(p ** 3 / 3.0 + p * p * q + p * q * q for p, q in cells)
    red = 0
    for g in F.levels[0].groups:
        c, k = g.c.size, g.sk.size
        assert g.skeletonized == (eps > 0 and k < c)
        if g.skeletonized:
            r = c - k
            cN = g.cN.size          # equals the closed form (multisets compared above)
            fl += 2.0 * cN * c * k + r ** 3 / 3.0 + 5.0 * k * r * r + 4.0 * k * k * r
            red += r
    top = n ** dim - sum(p for p, _ in cells) - red
    assert F.top_size == top
    fl += top ** 3 / 3.0
    assert OH.factor_flops(F) == pytest.approx(fl, rel=1e-12)
    if eps == 0.0:
        assert top == (2 * m) ** dim - (2 * m - 1) ** dim
