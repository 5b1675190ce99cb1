"""HIF-DE in plain FP64: Lemma 2.1, Lemma 2.2 / Corollary 2.3, Lemma 2.4 and
Algorithm 4.1, with the factored application of F^{-1} and F.

The active matrix ``A_l`` is kept as one global scipy sparse matrix together
with its structural pattern ``P`` (0/1, entries never dropped).  Neighbour
sets ``c^N`` (Section 2, notation) are read from ``P``: eliminating a cell
adds the clique ``c^N x c^N`` (the fill of Lemma 2.1), skeletonizing a group
removes its redundant unknowns and leaves a dense block on its skeleton.

Free choices fixed here (listed with their reasons in the design notes):

* Diagonal blocks are factored as ``L D L^T`` without pivoting, obtained from
  the Cholesky factor ``C`` as ``L = C diag(C)^-1``, ``D = diag(C)^2``.
* The ID is Householder QR with column pivoting; column norms are recomputed
  from the remaining rows at every step; among columns whose norm is within a
  relative ``tau`` of the largest, the one with the smallest original
  position wins; the rank ``k`` counts the leading steps with
  ``|R_jj| > eps |R_11|`` and stops at the first failure.
* Every ID of level l+1/2 is computed from ``A_{l+1/2}`` (before any group of
  that level is processed), elimination updates of a level are all formed
  from ``A_l``, and a group whose rank equals its size is left alone.
* ``eps = 0`` turns skeletonization off, which is the multifrontal method
  (Algorithm 3.1).
* With ``sketch=True`` (the randomized compression of Section 4.3) a group
  with ``|c^N| > |c| + 16`` takes the ID of ``Phi_c A_{c^N, c}``, ``Phi_c``
  the ``(|c| + 16) x |c^N|`` Gaussian matrix of ``oracle.philox`` for the
  group's level and key; the rank rule and tie-break are unchanged.

Pinned by: eps=0 reproduces a sparse direct solve (tests/test_oracle_hifde.py),
the block-diagonalizations of Lemmas 2.1 and 2.4 on random matrices, the ID
against LAPACK's pivoted QR and exact low-rank reconstruction, symmetry and
positive definiteness of F, the eigenvalue bound of Theorem 4.1's corollary,
the partition of the unknowns, e_a = O(eps), and the flop count against
closed-form sizes of the one-level tree; the sketched ID by its invariance
under orthogonal sketches, exact recovery of low-rank blocks and its error
against the deterministic ID (tests/test_oracle_sketch.py).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import philox, problem, tree


class NotSPD(RuntimeError):
    pass


# ---------------------------------------------------------------------------
# Dense primitives
# ---------------------------------------------------------------------------

def ldl_spd(A: np.ndarray):
    """Unpivoted ``A = L D L^T`` of an SPD block via its Cholesky factor."""
    if A.shape[0] == 0:
        return np.zeros((0, 0)), np.zeros(0)
    try:
        C = sla.cholesky(A, lower=True, check_finite=True)
    except sla.LinAlgError as exc:
        raise NotSPD(str(exc)) from exc
    d = np.diag(C).copy()
    return C / d[None, :], d * d


class Breakdown(RuntimeError):
    pass


def ldl_sym(A: np.ndarray, tiny: float = 1e-13):
    """Unpivoted ``A = L D L^T`` of a symmetric block that need not be
    definite (the indefinite problems of Section 5, Helmholtz-type
    ``b < 0`` at low frequency): column by column, ``D_j = A_jj - sum_k
    L_jk^2 D_k`` and ``L_ij = (A_ij - sum_k L_ik L_jk D_k) / D_j``.  A pivot
    with ``|D_j| <= tiny * max_i |A_ii|`` is a breakdown (no pivoting)."""
    n = A.shape[0]
    if n == 0:
        return np.zeros((0, 0)), np.zeros(0)
    L = np.eye(n)
    D = np.zeros(n)
    scale = float(np.max(np.abs(np.diag(A))))
    for j in range(n):
        D[j] = A[j, j] - np.sum(L[j, :j] ** 2 * D[:j])
        if not abs(D[j]) > tiny * scale:
            raise Breakdown(f"pivot {j} of an unpivoted LDL^T is {D[j]:.3e}")
        L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ (L[j, :j] * D[:j])) / D[j]
    return L, D


def _ldl(A: np.ndarray, definite: bool):
    return ldl_spd(A) if definite else ldl_sym(A)


def sparse_elimination(App: np.ndarray, Aqp: np.ndarray, definite: bool = True):
    """Lemma 2.1: ``A_pp = L D L^T``; ``W = D^-1 L^-1 A_qp^T`` is the
    off-diagonal block of the elimination operator ``S_p``; the Schur
    complement update on the front is ``-A_qp A_pp^-1 A_qp^T``.

    Returns ``(L, D, W, update)``."""
    L, D = _ldl(App, definite)
    if Aqp.shape[0] == 0:
        return L, D, np.zeros((App.shape[0], 0)), np.zeros((0, 0))
    Y = sla.solve_triangular(L, Aqp.T, lower=True, unit_diagonal=True)   # L^-1 A_pq
    W = Y / D[:, None]
    update = -(Y.T @ W)                                                    # -A_qp L^-T D^-1 L^-1 A_pq
    return L, D, W, 0.5 * (update + update.T)


@dataclass
class IDResult:
    k: int
    perm: np.ndarray        # column order: skeletons (pivot order) then redundant
    T: np.ndarray           # k x (n-k), in pivot order
    rdiag: np.ndarray       # |R_jj| of the accepted steps
    norms_at_stop: Optional[np.ndarray] = None


def interp_decomp(M: np.ndarray, eps: float, tau: float = 1e-10) -> IDResult:
    """Adaptive-rank ID by column-pivoted Householder QR (Section 2.2).

    ``M[:, perm[k:]] ~= M[:, perm[:k]] @ T``.  ``eps <= 0`` is not allowed here
    (the caller treats eps = 0 as "no skeletonization")."""
    m, n = M.shape
    R = np.array(M, dtype=np.float64, copy=True)
    perm = np.arange(n)
    rdiag = []
    k = 0
    ref = 0.0
    for j in range(min(m, n)):
        norms = np.sqrt(np.sum(R[j:, j:] ** 2, axis=0))
        mx = norms.max()
        cand = np.nonzero(norms >= (1.0 - tau) * mx)[0]
        sel = int(cand[np.argmin(perm[j + cand])])
        rjj = float(norms[sel])
        if j == 0:
            ref = rjj
            if ref == 0.0:
                break
        if not rjj > eps * ref:
            break
        piv = j + sel
        if piv != j:
            R[:, [j, piv]] = R[:, [piv, j]]
            perm[[j, piv]] = perm[[piv, j]]
        x = R[j:, j].copy()
        alpha = -np.copysign(np.linalg.norm(x), x[0] if x[0] != 0 else 1.0)
        v = x
        v[0] -= alpha
        vn = float(v @ v)
        if vn > 0.0:
            R[j:, j:] -= np.outer(v, (2.0 / vn) * (v @ R[j:, j:]))
        R[j + 1:, j] = 0.0
        rdiag.append(rjj)
        k += 1
    if k > 0 and k < n:
        T = sla.solve_triangular(R[:k, :k], R[:k, k:], lower=False)
    else:
        T = np.zeros((k, n - k))
    return IDResult(k, perm, T, np.array(rdiag))


def skeletonize_block(Arr, Asr, Ass, T, definite: bool = True):
    """Lemma 2.4 on a group ``c = (r, s)`` with ``A_{:,r} ~= A_{:,s} T``:
    ``B_rr = A_rr - T^T A_sr - A_sr^T T + T^T A_ss T``, ``B_sr = A_sr - A_ss T``,
    ``B_rr = L_r D_r L_r^T``, ``W_r = D_r^-1 L_r^-1 B_sr^T`` and the new skeleton
    block ``B_ss = A_ss - B_sr B_rr^-1 B_sr^T``.

    Returns ``(L_r, D_r, W_r, B_ss)``."""
    Brr = Arr - T.T @ Asr - Asr.T @ T + T.T @ Ass @ T
    Brr = 0.5 * (Brr + Brr.T)
    Bsr = Asr - Ass @ T
    Lr, Dr = _ldl(Brr, definite)
    Y = sla.solve_triangular(Lr, Bsr.T, lower=True, unit_diagonal=True)
    Wr = Y / Dr[:, None]
    Bss = Ass - Y.T @ Wr
    return Lr, Dr, Wr, 0.5 * (Bss + Bss.T)


# ---------------------------------------------------------------------------
# Factor containers
# ---------------------------------------------------------------------------

@dataclass
class CellFactor:
    cid: int
    p: np.ndarray
    q: np.ndarray
    L: np.ndarray
    D: np.ndarray
    W: np.ndarray


@dataclass
class GroupFactor:
    gid: int
    c: np.ndarray
    cN: np.ndarray
    sk: np.ndarray           # sorted skeleton unknowns
    rd: np.ndarray           # sorted redundant unknowns
    T: np.ndarray            # |sk| x |rd|, rows/cols in sorted order
    Lr: np.ndarray
    Dr: np.ndarray
    Wr: np.ndarray
    skeletonized: bool
    rdiag: np.ndarray = field(default_factory=lambda: np.zeros(0))


@dataclass
class Level:
    cells: List[CellFactor] = field(default_factory=list)
    groups: List[GroupFactor] = field(default_factory=list)


@dataclass
class Factor:
    dim: int
    n: int
    m: int
    L: int
    eps: float
    N: int
    levels: List[Level]
    top: CellFactor
    A: sp.csr_matrix

    @property
    def top_size(self) -> int:
        return int(self.top.p.size)


# ---------------------------------------------------------------------------
# Global bookkeeping
# ---------------------------------------------------------------------------

def _sub(A: sp.csr_matrix, r: np.ndarray, c: np.ndarray) -> np.ndarray:
    if r.size == 0 or c.size == 0:
        return np.zeros((r.size, c.size))
    return A[r][:, c].toarray()


def _neighbors(P: sp.csr_matrix, c: np.ndarray) -> np.ndarray:
    """``c^N``: unknowns outside ``c`` coupled to ``c`` in the pattern."""
    cols = np.unique(P[c].indices)
    return np.setdiff1d(cols, c, assume_unique=True)


def _mask(A: sp.csr_matrix, keep: np.ndarray) -> sp.csr_matrix:
    Dm = sp.diags(keep.astype(np.float64))
    out = (Dm @ A @ Dm).tocsr()
    out.eliminate_zeros()
    out.sort_indices()
    return out


def _add_blocks(A: sp.csr_matrix, blocks) -> sp.csr_matrix:
    if not blocks:
        return A
    rows, cols, vals = [], [], []
    for idx, V in blocks:
        rr, cc = np.meshgrid(idx, idx, indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(np.asarray(V).ravel())
    U = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=A.shape).tocsr()
    out = (A + U).tocsr()
    out.sort_indices()
    return out


# ---------------------------------------------------------------------------
# Algorithm 4.1
# ---------------------------------------------------------------------------

def factor(dim: int, n: int, m: int, a, b=None, eps: float = 1e-6,
           skip_levels: int = 0, tau: float = 1e-10, definite: bool = True,
           sketch: bool = False) -> Factor:
    """HIF-DE factorization ``A ~= V_0^-T ... V_{L-1/2}^-T D V_{L-1/2}^-1 ... V_0^-1``.

    ``definite=False`` factors every diagonal block by the unpivoted
    ``ldl_sym`` (negative pivots allowed): F is then a congruence of the
    block-diagonal D, symmetric but indefinite, for GMRES (Section 5).
    ``sketch=True`` compresses ``Phi_c A_{c^N, c}`` instead of
    ``A_{c^N, c}`` where ``|c^N| > |c| + 16`` (Section 4.3, randomized ID)."""
    if eps < 0 or eps >= 1:
        raise ValueError("eps must lie in [0, 1)")
    L = tree.num_levels(n, m)
    A0 = problem.assemble(dim, n, a, b)
    A = A0.copy()
    P = problem.stencil_pattern(A0)
    coords = problem.dof_coords(dim, n)
    N = n ** dim
    active = np.ones(N, dtype=bool)
    levels: List[Level] = []
    for lvl in range(L):
        lev = Level()
        # -- level l: eliminate interior cells (Lemma 2.1 on every c in C_l)
        upd, cliques = [], []
        for cid, p in tree.cells_at_level(coords, active, n, m, lvl):
            q = _neighbors(P, p)
            App = _sub(A, p, p)
            Aqp = _sub(A, q, p)
            Lc, Dc, Wc, U = sparse_elimination(App, Aqp, definite)
            lev.cells.append(CellFactor(cid, p, q, Lc, Dc, Wc))
            if q.size:
                upd.append((q, U))
                cliques.append((q, np.ones((q.size, q.size))))
            active[p] = False
        A = _mask(_add_blocks(A, upd), active)
        P = _mask(_add_blocks(P, cliques), active)
        # -- level l+1/2: skeletonize edges (2D) / faces (3D) (Lemma 2.4)
        deltas, cliques, removed = [], [], []
        for gid, c in tree.groups_at_level(coords, active, n, m, lvl):
            cN = _neighbors(P, c)
            do_skel = eps > 0 and lvl >= skip_levels
            if do_skel:
                Mblk = _sub(A, cN, c)
                rows = philox.sketch_rows(c.size, cN.size)
                if sketch and rows < cN.size:
                    Mblk = philox.sketch_matrix(lvl, int(gid), rows, cN.size) @ Mblk
                idr = interp_decomp(Mblk, eps, tau)
                k = idr.k
                if k == c.size:
                    do_skel = False
            if not do_skel:
                lev.groups.append(GroupFactor(gid, c, cN, c.copy(), c[:0].copy(),
                                              np.zeros((c.size, 0)), np.zeros((0, 0)),
                                              np.zeros(0), np.zeros((0, c.size)), False))
                continue
            perm = idr.perm
            sk_pos = np.sort(perm[:k])
            rd_pos = np.sort(perm[k:])
            # T rows follow the pivot order of perm[:k]; reorder both ways
            row_order = np.argsort(perm[:k])
            col_order = np.argsort(perm[k:])
            T = idr.T[row_order][:, col_order]
            Acc = _sub(A, c, c)
            Arr = Acc[np.ix_(rd_pos, rd_pos)]
            Asr = Acc[np.ix_(sk_pos, rd_pos)]
            Ass = Acc[np.ix_(sk_pos, sk_pos)]
            Lr, Dr, Wr, Bss = skeletonize_block(Arr, Asr, Ass, T, definite)
            sk, rd = c[sk_pos], c[rd_pos]
            lev.groups.append(GroupFactor(gid, c, cN, sk, rd, T, Lr, Dr, Wr, True, idr.rdiag))
            deltas.append((sk, Bss - Ass))
            cliques.append((sk, np.ones((sk.size, sk.size))))
            removed.append(rd)
        for rd in removed:
            active[rd] = False
        A = _mask(_add_blocks(A, deltas), active)
        P = _mask(_add_blocks(P, cliques), active)
        levels.append(lev)
    # -- level L: the remaining block D on s_L
    sL = np.nonzero(active)[0]
    Ltop, Dtop = _ldl(_sub(A, sL, sL), definite)
    top = CellFactor(-1, sL, sL[:0].copy(), Ltop, Dtop, np.zeros((sL.size, 0)))
    return Factor(dim, n, m, L, eps, N, levels, top, A0)


# ---------------------------------------------------------------------------
# Application of F^{-1} and F in factored form
# ---------------------------------------------------------------------------

def _tri(L, X, trans=False):
    return sla.solve_triangular(L, X, lower=True, unit_diagonal=True, trans=1 if trans else 0)


def solve(F: Factor, f: np.ndarray) -> np.ndarray:
    """``F^-1 f = V_0 V_{1/2} ... D^-1 ... V_{1/2}^T V_0^T f``."""
    x = np.array(f, dtype=np.float64, copy=True)
    vec = x.ndim == 1
    if vec:
        x = x[:, None]
    # upward: V_0^T, V_{1/2}^T, ...
    for lev in F.levels:
        for c in lev.cells:
            xp = _tri(c.L, x[c.p])
            x[c.p] = xp
            if c.q.size:
                x[c.q] -= c.W.T @ xp
        for g in lev.groups:
            if not g.skeletonized:
                continue
            x[g.rd] -= g.T.T @ x[g.sk]                 # Q^T
            xr = _tri(g.Lr, x[g.rd])                   # S_r^T
            x[g.rd] = xr
            x[g.sk] -= g.Wr.T @ xr
    # D^-1
    for lev in F.levels:
        for c in lev.cells:
            x[c.p] /= c.D[:, None]
        for g in lev.groups:
            if g.skeletonized:
                x[g.rd] /= g.Dr[:, None]
    t = F.top
    if t.p.size:
        x[t.p] = _tri(t.L, _tri(t.L, x[t.p]) / t.D[:, None], trans=True)
    # downward: ..., V_{1/2}, V_0
    for lev in reversed(F.levels):
        for g in lev.groups:
            if not g.skeletonized:
                continue
            x[g.rd] = _tri(g.Lr, x[g.rd] - g.Wr @ x[g.sk], trans=True)   # S_r
            x[g.sk] -= g.T @ x[g.rd]                                        # Q
        for c in lev.cells:
            rhs = x[c.p] - (c.W @ x[c.q] if c.q.size else 0.0)
            x[c.p] = _tri(c.L, rhs, trans=True)
    return x[:, 0] if vec else x


def apply(F: Factor, v: np.ndarray) -> np.ndarray:
    """``F v = V_0^-T ... D ... V_0^-1 v``; each elementary factor is inverted
    by negating its off-diagonal block (Section 3.1)."""
    x = np.array(v, dtype=np.float64, copy=True)
    vec = x.ndim == 1
    if vec:
        x = x[:, None]
    # V_0^-1, V_{1/2}^-1, ...   (S^-1 = [[L^T, W], [0, I]], Q^-1 adds T)
    for lev in F.levels:
        for c in lev.cells:
            xp = c.L.T @ x[c.p]
            if c.q.size:
                xp = xp + c.W @ x[c.q]
            x[c.p] = xp
        for g in lev.groups:
            if not g.skeletonized:
                continue
            x[g.sk] += g.T @ x[g.rd]                          # Q^-1
            x[g.rd] = g.Lr.T @ x[g.rd] + g.Wr @ x[g.sk]       # S_r^-1
    for lev in F.levels:
        for c in lev.cells:
            x[c.p] *= c.D[:, None]
        for g in lev.groups:
            if g.skeletonized:
                x[g.rd] *= g.Dr[:, None]
    t = F.top
    if t.p.size:
        x[t.p] = t.L @ (t.D[:, None] * (t.L.T @ x[t.p]))
    # ..., V_{1/2}^-T, V_0^-T   (S^-T = [[L, 0], [W^T, I]], Q^-T adds T^T)
    for lev in reversed(F.levels):
        for g in lev.groups:
            if not g.skeletonized:
                continue
            xr = x[g.rd]
            x[g.sk] += g.Wr.T @ xr
            x[g.rd] = g.Lr @ xr
            x[g.rd] += g.T.T @ x[g.sk]
        for c in lev.cells:
            xp = x[c.p]
            if c.q.size:
                x[c.q] += c.W.T @ xp
            x[c.p] = c.L @ xp
    return x[:, 0] if vec else x


# ---------------------------------------------------------------------------
# Index sets and statistics
# ---------------------------------------------------------------------------

def export_sets(F: Factor):
    """Per level: cells ``(cid, p, q)`` and groups ``(gid, c, cN, sk, rd)``."""
    out = []
    for lev in F.levels:
        out.append({
            "cells": [(c.cid, c.p, c.q) for c in lev.cells],
            "groups": [(g.gid, g.c, g.cN, g.sk, g.rd) for g in lev.groups],
        })
    return out, F.top.p


def partition_sizes(F: Factor) -> int:
    """``sum |p| + sum |r| + |s_L|``; equals N when every unknown is
    eliminated exactly once (the block partition theta_L)."""
    tot = F.top.p.size
    for lev in F.levels:
        tot += sum(c.p.size for c in lev.cells)
        tot += sum(g.rd.size for g in lev.groups)
    return int(tot)


def factor_flops(F: Factor) -> float:
    """Algorithmic flop count of the factorization (dense-block model):
    cells ``p^3/3 + p^2 q + p q^2`` (Lemma 2.1: the LDL^T of A_pp, W and the
    Schur update of the front); skeletonized groups
    ``2|c^N||c|k + r^3/3 + 5 k r^2 + 4 k^2 r`` (the ID of Section 2.2 and
    Lemma 2.4's B_rr, B_sr, LDL^T and update); top ``|s_L|^3/3``.  A group
    that keeps all of ``c`` (k = |c|, or no ID at eps = 0 and on skipped
    levels) is left alone and counts nothing."""
    fl = F.top.p.size ** 3 / 3.0
    for lev in F.levels:
        for c in lev.cells:
            p, q = c.p.size, c.q.size
            fl += p ** 3 / 3.0 + p * p * q + p * q * q
        for g in lev.groups:
            if not g.skeletonized:
                continue
            k, r = g.sk.size, g.rd.size
            fl += 2.0 * g.cN.size * g.c.size * k + r ** 3 / 3.0 + 5.0 * k * r * r + 4.0 * k * k * r
    return fl
