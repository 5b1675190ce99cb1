"""Cells, separators and skeletonization groups of the uniform tree.

Geometry (Sections 3.1, 4.1, 4.2): at level l the domain is cut into boxes of
``M_l = m 2^l`` unknowns per side, ``B_l = ceil(n / M_l)`` of them along each
axis; the last box along an axis is shorter when ``M_l`` does not divide
``n`` (any ``n`` with at least two leaf boxes per side; ``n = m 2^L`` gives
the uniform tree of the paper's figures, ``n = 2^k - 1`` its example grids).
The separators are the last row of every box but the last along each axis:
coordinate ``x_k`` lies on a level-l separator iff ``(x_k + 1) mod M_l == 0``
and ``x_k != n-1``.  The top level L is the first with a single box
(``m 2^L >= n``).

* ``sigma_l(i)`` counts the axes on which unknown ``i`` lies on a level-l
  separator.
* Level-l cells (the collection C_l): active unknowns with ``sigma_l = 0``,
  grouped by their box ``floor(x / M_l)``.
* Level-(l+1/2) groups (C_{l+1/2}): active unknowns with ``sigma_l = 1`` -- the
  Voronoi cells about edge centres (2D) or face centres (3D) -- keyed by the
  separator axis, the plane index ``floor(x_k / M_l)`` and the box indices of
  the other axes.  Unknowns with ``sigma_l >= 2`` (corner points in 2D,
  corner edges in 3D) belong to no group (Section 4.3, "not at all").

Pinned by counting identities (number of cells and groups per level, number
of level-0 separator unknowns) in tests/test_oracle_tree.py.
"""
from __future__ import annotations

import numpy as np


def boxes(n: int, M: int) -> int:
    """Boxes of side M along an axis of n unknowns (the last may be short)."""
    return -(-n // M)


def num_levels(n: int, m: int) -> int:
    if m < 2:
        raise ValueError("leaf size must be >= 2")
    B0 = boxes(n, m)
    if B0 < 2:
        raise ValueError("n must hold at least two leaf boxes per side")
    L = 0
    while (1 << L) < B0:
        L += 1
    return L


def sep_axis(n: int, M: int) -> np.ndarray:
    x = np.arange(n)
    return ((x + 1) % M == 0) & (x != n - 1)


def sigma(coords: np.ndarray, n: int, M: int) -> np.ndarray:
    s = sep_axis(n, M)
    return s[coords].sum(axis=1)


def box_id(coords: np.ndarray, n: int, M: int) -> np.ndarray:
    """Lexicographic box index (x0 fastest) of each unknown at box side M."""
    B = boxes(n, M)
    bx = coords // M
    out = np.zeros(coords.shape[0], dtype=np.int64)
    for k in range(coords.shape[1]):
        out += bx[:, k] * B ** k
    return out


def group_id(coords: np.ndarray, n: int, M: int) -> np.ndarray:
    """Key of the group holding each sigma=1 unknown:
    ``k * B^d + lexicographic(box indices with box_k := plane index)``."""
    dim = coords.shape[1]
    B = boxes(n, M)
    s = sep_axis(n, M)[coords]                     # (N, dim) bool
    k = np.argmax(s, axis=1)
    bx = coords // M
    out = k.astype(np.int64) * B ** dim
    for j in range(dim):
        out += bx[:, j] * B ** j
    return out


def cells_at_level(coords, active, n, m, level):
    """Sorted list of (cell_id, p) with p the sorted active interior unknowns."""
    M = m << level
    sig = sigma(coords, n, M)
    sel = np.nonzero(active & (sig == 0))[0]
    bid = box_id(coords[sel], n, M)
    order = np.lexsort((sel, bid))
    sel, bid = sel[order], bid[order]
    out = []
    if sel.size:
        cuts = np.nonzero(np.diff(bid))[0] + 1
        for part_idx, part_box in zip(np.split(sel, cuts), np.split(bid, cuts)):
            out.append((int(part_box[0]), part_idx))
    return out


def groups_at_level(coords, active, n, m, level):
    """Sorted list of (group_id, c) for the level-(level+1/2) groups."""
    M = m << level
    sig = sigma(coords, n, M)
    sel = np.nonzero(active & (sig == 1))[0]
    gid = group_id(coords[sel], n, M)
    order = np.lexsort((sel, gid))
    sel, gid = sel[order], gid[order]
    out = []
    if sel.size:
        cuts = np.nonzero(np.diff(gid))[0] + 1
        for part_idx, part_g in zip(np.split(sel, cuts), np.split(gid, cuts)):
            out.append((int(part_g[0]), part_idx))
    return out
