"""Shared helpers for the GPU parity tests: run the oracle and the HIP path
on the same seeded inputs and compare index sets and residuals."""
from __future__ import annotations

import numpy as np

from oracle import hifde as OH
from synth import workloads as W


def oracle_factor(dim, n, m, a, eps, skip=0):
    return OH.factor(dim, n, m, a, eps=eps, skip_levels=skip)


def torch_inputs(a, device="cuda"):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(device) for x in a]


def gpu_factor(dim, n, m, a, eps, prec, skip=0):
    import paper_1307_2895_amd as H
    T = H.hifde_build_tree(dim, n, m, skip)
    F = H.hifde_factor(T, torch_inputs(a), None, eps, prec)
    return T, F


def compare_sets(OF, F, check_skeletons=True):
    """Compare every level's index sets; returns (n_cell_mismatch,
    n_group_struct_mismatch, n_skeleton_mismatch, first_skeleton_level)."""
    import paper_1307_2895_amd as H
    sets, top = OH.export_sets(OF)
    cm = gm = sm = 0
    first = None
    for l, lev in enumerate(sets):
        gc = H.hifde_export_sets(F, 2 * l)
        if len(gc) != len(lev["cells"]):
            return (10 ** 9, 0, 0, l)
        for (cid, p, q), (hid, hl) in zip(lev["cells"], gc):
            if cid != hid or not np.array_equal(p, hl[0]) or not np.array_equal(q, hl[1]):
                cm += 1
        gg = H.hifde_export_sets(F, 2 * l + 1)
        if len(gg) != len(lev["groups"]):
            return (cm, 10 ** 9, 0, l)
        for (gid, c, cN, sk, rd), (hid, hl) in zip(lev["groups"], gg):
            if gid != hid or not np.array_equal(c, hl[0]) or not np.array_equal(cN, hl[1]):
                gm += 1
            if not (np.array_equal(sk, hl[2]) and np.array_equal(rd, hl[3])):
                sm += 1
                if first is None:
                    first = l
    tp = H.hifde_export_sets(F, 2 * OF.L)
    if not np.array_equal(tp[0][1][0], top):
        cm += 1
    return cm, gm, sm, first


def compare_structure(OF, F, levels):
    """Cells (p, c^N) of levels < ``levels`` and groups (c, c^N) of levels
    l + 1/2 < ``levels``: the sets that no skeleton choice of those levels
    changes.  Returns (cell mismatches, group mismatches)."""
    import paper_1307_2895_amd as H
    sets, _ = OH.export_sets(OF)
    cm = gm = 0
    for l in range(levels):
        lev = sets[l]
        gc = H.hifde_export_sets(F, 2 * l)
        if len(gc) != len(lev["cells"]):
            return 10 ** 9, 0
        for (cid, p, q), (hid, hl) in zip(lev["cells"], gc):
            if cid != hid or not np.array_equal(p, hl[0]) or not np.array_equal(q, hl[1]):
                cm += 1
        gg = H.hifde_export_sets(F, 2 * l + 1)
        if len(gg) != len(lev["groups"]):
            return cm, 10 ** 9
        for (gid, c, cN, _, _), (hid, hl) in zip(lev["groups"], gg):
            if gid != hid or not np.array_equal(c, hl[0]) or not np.array_equal(cN, hl[1]):
                gm += 1
    return cm, gm


def rel_residual(A, u, f):
    r = f - A @ u
    return np.linalg.norm(r, axis=0) / np.linalg.norm(f, axis=0)
