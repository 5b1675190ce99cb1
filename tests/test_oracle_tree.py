"""Pins of the tree geometry by counting identities (Sections 3.1, 4.1, 4.2)."""
import numpy as np
import pytest

from oracle import hifde as OH
from oracle import problem, tree
from synth import workloads as W


@pytest.mark.parametrize("dim,n,m", [(2, 64, 8), (2, 48, 3), (3, 16, 4), (3, 32, 4)])
def test_level0_counts(dim, n, m):
    L = tree.num_levels(n, m)
    B0 = n // m
    X = problem.dof_coords(dim, n)
    active = np.ones(n ** dim, dtype=bool)
    cells = tree.cells_at_level(X, active, n, m, 0)
    assert len(cells) == 2 ** (dim * L)
    # separator unknowns: everything outside the cell interiors
    n_int = sum(len(p) for _, p in cells)
    assert n ** dim - n_int == n ** dim - ((B0 - 1) * (m - 1) + m) ** dim
    for _, p in cells:
        active[p] = False
    groups = tree.groups_at_level(X, active, n, m, 0)
    if dim == 2:
        assert len(groups) == 2 * B0 * (B0 - 1)
    else:
        assert len(groups) == 3 * (B0 - 1) * B0 ** 2


def test_config_counts():
    """The 2D Laplacian workload has 847 level-0 separator unknowns and 112
    level-1/2 edges; the 3D n=64 workload 144495 and 11520 faces."""
    for dim, n, m, nsep, ngrp in [(2, 64, 8, 847, 112), (3, 64, 4, 144495, 11520)]:
        B0 = n // m
        assert n ** dim - ((B0 - 1) * (m - 1) + m) ** dim == nsep
        assert (2 * B0 * (B0 - 1) if dim == 2 else 3 * (B0 - 1) * B0 ** 2) == ngrp


@pytest.mark.parametrize("dim,n,m,eps", [(2, 32, 4, 1e-6), (2, 48, 3, 1e-3), (3, 16, 2, 1e-6), (3, 16, 4, 0.0)])
def test_partition_invariant(dim, n, m, eps):
    """Every unknown is eliminated exactly once: sum |p| + sum |r| + |s_L| = N
    (the block partition theta_L of Section 4.1)."""
    a = W.make_field(dim, n, "loguniform", 9)
    F = OH.factor(dim, n, m, a, eps=eps)
    assert OH.partition_sizes(F) == n ** dim
    seen = np.zeros(n ** dim, dtype=int)
    for lev in F.levels:
        for c in lev.cells:
            seen[c.p] += 1
        for g in lev.groups:
            seen[g.rd] += 1
    seen[F.top.p] += 1
    assert np.all(seen == 1)


def test_corners_never_grouped():
    """Unknowns on two or more separators (2D corners, 3D corner edges) are
    in no group at that level (Section 4.3)."""
    n, m = 32, 4
    for dim in (2, 3):
        X = problem.dof_coords(dim, n)
        active = np.ones(n ** dim, dtype=bool)
        for _, p in tree.cells_at_level(X, active, n, m, 0):
            active[p] = False
        sig = tree.sigma(X, n, m)
        grouped = np.zeros(n ** dim, dtype=bool)
        for _, c in tree.groups_at_level(X, active, n, m, 0):
            grouped[c] = True
        assert not np.any(grouped & (sig >= 2))
        assert np.all(grouped[active & (sig == 1)])


# Grids whose side is not m 2^L: the last box along each axis is short.
RAGGED = [(2, 60, 8), (2, 65, 8), (3, 30, 4), (2, 1023, 16)]


@pytest.mark.parametrize("dim,n,m", RAGGED)
def test_ragged_counts(dim, n, m):
    """B_l = ceil(n / (m 2^l)) boxes per axis; each box keeps its non-separator
    coordinates (n - (B_0 - 1) per axis in all), the level-1/2 groups are the
    (B_0 - 1) separator planes times the boxes of the other axes, and the
    top level L is the first with one box."""
    L = tree.num_levels(n, m)
    B0 = -(-n // m)
    assert (m << (L - 1)) < n <= (m << L)
    X = problem.dof_coords(dim, n)
    active = np.ones(n ** dim, dtype=bool)
    cells = tree.cells_at_level(X, active, n, m, 0)
    assert len(cells) == B0 ** dim
    assert sum(len(p) for _, p in cells) == (n - (B0 - 1)) ** dim
    for _, p in cells:
        active[p] = False
    groups = tree.groups_at_level(X, active, n, m, 0)
    if dim == 2:
        assert len(groups) == 2 * B0 * (B0 - 1)
    else:
        assert len(groups) == 3 * (B0 - 1) * B0 ** 2
    assert not np.any(tree.sep_axis(n, m << L))


@pytest.mark.parametrize("dim,n,m,eps", [(2, 60, 8, 1e-6), (2, 65, 8, 1e-3), (3, 30, 4, 1e-6)])
def test_ragged_partition_and_exact_solve(dim, n, m, eps):
    """Every unknown is eliminated once on ragged grids, and at eps = 0 the
    factorization is a sparse direct solve."""
    import scipy.sparse.linalg as spla
    a = W.make_field(dim, n, "loguniform", 9)
    F = OH.factor(dim, n, m, a, eps=eps)
    assert OH.partition_sizes(F) == n ** dim
    F0 = OH.factor(dim, n, m, a, eps=0.0)
    f = W.make_rhs(n ** dim, 1, 4)[:, 0]
    ud = spla.spsolve(F0.A.tocsc(), f)
    assert np.linalg.norm(OH.solve(F0, f) - ud) <= 1e-11 * np.linalg.norm(ud)
