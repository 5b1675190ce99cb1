"""HIF-DE (hierarchical interpolative factorization for elliptic PDEs) on
AMD MI355X (gfx950).

The Python functions mirror the C ABI of ``include/hifde.h`` one to one and
only marshal arguments; the factorization, F^-1 sweeps, PCG and GMRES run in the
HIP library ``libhifde.so``.  torch supplies device memory and the stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from ._lib import (  # noqa: F401
    HIFDE_FP64, HIFDE_MIXED, HIFDE_MIXED_ELIM64, HIFDE_DEBUG_DETERMINISM, HIFDE_NO_GRAPH, HIFDE_USE_RANK_MODEL,
    HIFDE_AUTOTUNE,
    HIFDE_PRESIZE_WORST_CASE, HIFDE_SWEEP_ROW_TILES, HIFDE_INDEFINITE, HIFDE_SKETCH_ID,
    HIFDE_RETRY_FP64,
    HifdeError, Prof, Sets, Stats, check, lib,
    HIFDE_ENOCONV, HIFDE_EINVAL, HIFDE_ENOTSPD, HIFDE_ESTATE, HIFDE_ENOMEM,
    HIFDE_PROF_SWEEP_UP, HIFDE_PROF_SWEEP_DOWN, HIFDE_PROF_INTERP, HIFDE_PROF_TOP,
    HIFDE_PROF_SWEEP_UP_WHOLE, HIFDE_PROF_SWEEP_DOWN_WHOLE, HIFDE_PROF_GROUP_UP,
    HIFDE_PROF_GROUP_DOWN, HIFDE_PROF_SWEEP_UP_ONE, HIFDE_PROF_CONTRIB_ADD,
    HIFDE_PROF_CLASSES, HIFDE_RANK_FEATURES, HIFDE_RANK_HIDDEN, HIFDE_RANK_PARAMS,
    HIFDE_MLP_NOALLOC_MAX_BATCH,
)


# Workload precision names -> hifde_precision.
PRECISIONS = {"fp64": HIFDE_FP64, "mixed": HIFDE_MIXED, "mixed_elim64": HIFDE_MIXED_ELIM64}


class Tree:
    def __init__(self, handle, dim, n, leaf, skip):
        self._h = handle
        self.dim, self.n, self.leaf, self.skip = dim, n, leaf, skip
        self.N = n ** dim

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().hifde_tree_free(self._h)
                self._h = None
        except Exception:  # interpreter shutdown: the library may be gone
            pass


class Factor:
    def __init__(self, handle, tree, prec=None):
        self._h = handle
        self.tree = tree
        self.prec = prec

    @property
    def N(self):
        return self.tree.N

    def free(self):
        if getattr(self, "_h", None):
            lib().hifde_factor_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:  # interpreter shutdown: the library may be gone
            pass


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def hifde_build_tree(dim: int, n: int, leaf: int, skip_levels: int = 0) -> Tree:
    h = C.c_void_p()
    check(lib().hifde_build_tree(dim, n, leaf, skip_levels, C.byref(h)))
    return Tree(h, dim, n, leaf, skip_levels)


def hifde_tree_set_memory_limit(tree: Tree, nbytes: int):
    """Cap (bytes, 0 = none) on the device memory the tree's factorizations
    and solves may hold; exceeding it gives HIFDE_ENOMEM."""
    check(lib().hifde_tree_set_memory_limit(tree._h, int(nbytes)))


def hifde_factor(tree: Tree, a, b=None, eps: float = 1e-6, prec: int = HIFDE_FP64,
                 flags: int = 0, stream=None) -> Factor:
    """``a``: list of ``dim`` float64 CUDA tensors (link coefficients, C-order
    shapes as in ``include/hifde.h``); ``b``: float64 CUDA tensor of N or None."""
    for t in a:
        if not (t.is_cuda and t.is_contiguous() and str(t.dtype) == "torch.float64"):
            raise HifdeError(-1, "a[k] must be contiguous float64 CUDA tensors")
    arr = (C.c_void_p * tree.dim)(*[t.data_ptr() for t in a])
    bp = C.c_void_p(b.data_ptr()) if b is not None else C.c_void_p()
    h = C.c_void_p()
    check(lib().hifde_factor(tree._h, arr, bp, float(eps), int(prec), int(flags),
                             _stream(stream), C.byref(h)))
    return Factor(h, tree, prec)


def _as_colmajor(f, N):
    """(N,) or (N, nrhs) tensor -> contiguous (nrhs, N) tensor (= N x nrhs
    column-major) and the original shape."""
    if f.dim() == 1:
        return f.reshape(1, N).contiguous(), (N,)
    return f.t().contiguous(), tuple(f.shape)


def hifde_solve(F: Factor, f, stream=None):
    """u = F^-1 f for a float64 CUDA tensor of shape (N,) or (N, nrhs)."""
    import torch
    N = F.N
    fc, shape = _as_colmajor(f, N)
    nrhs = fc.shape[0]
    u = torch.empty_like(fc)
    check(lib().hifde_solve(F._h, nrhs, _dptr(fc), N, _dptr(u), N, _stream(stream)))
    return u.reshape(shape) if len(shape) == 1 else u.t()


def hifde_matvec(F: Factor, x, stream=None):
    import torch
    N = F.N
    xc, shape = _as_colmajor(x, N)
    nrhs = xc.shape[0]
    y = torch.empty_like(xc)
    check(lib().hifde_matvec(F._h, nrhs, _dptr(xc), N, _dptr(y), N, _stream(stream)))
    return y.reshape(shape) if len(shape) == 1 else y.t()


def hifde_pcg(F: Factor, f, tol: float = 1e-12, maxit: int = 200, stream=None,
              raise_on_noconv: bool = True):
    """PCG with preconditioner F^-1.  Returns ``(u, iters, relres)``."""
    import torch
    N = F.N
    fc, shape = _as_colmajor(f, N)
    nrhs = fc.shape[0]
    u = torch.empty_like(fc)
    its = (C.c_int * nrhs)()
    rel = (C.c_double * nrhs)()
    rc = lib().hifde_pcg(F._h, nrhs, _dptr(fc), N, _dptr(u), N, float(tol), int(maxit), its, rel,
                         _stream(stream))
    if rc != 0 and (raise_on_noconv or rc != HIFDE_ENOCONV):
        check(rc)
    out = u.reshape(shape) if len(shape) == 1 else u.t()
    return out, np.array(its[:]), np.array(rel[:])


def hifde_gmres(F: Factor, f, tol: float = 1e-12, restart: int = 30, maxit: int = 200,
                stream=None, raise_on_noconv: bool = True):
    """Restarted GMRES with right preconditioner F^-1.  Returns
    ``(u, iters, relres)``."""
    import torch
    N = F.N
    fc, shape = _as_colmajor(f, N)
    nrhs = fc.shape[0]
    u = torch.empty_like(fc)
    its = (C.c_int * nrhs)()
    rel = (C.c_double * nrhs)()
    rc = lib().hifde_gmres(F._h, nrhs, _dptr(fc), N, _dptr(u), N, float(tol), int(restart),
                           int(maxit), its, rel, _stream(stream))
    if rc != 0 and (raise_on_noconv or rc != HIFDE_ENOCONV):
        check(rc)
    out = u.reshape(shape) if len(shape) == 1 else u.t()
    return out, np.array(its[:]), np.array(rel[:])


def hifde_stats(F: Factor) -> dict:
    s = Stats()
    check(lib().hifde_stats(F._h, C.byref(s)))
    L = s.levels
    return {
        "N": s.N, "dim": s.dim, "levels": L, "top_size": s.top_size,
        "factor_bytes": s.factor_bytes, "factor_flops": s.factor_flops,
        "factor_ms": s.factor_ms, "solve_bytes": s.solve_bytes,
        "cells": list(s.cells[:L + 1]), "groups": list(s.groups[:L]),
        "skel_in": list(s.skel_in[:L]), "skel_out": list(s.skel_out[:L]),
        "max_front": list(s.max_front[:L + 1]),
        "rank_groups": s.rank_groups, "rank_mae": s.rank_mae, "rebuckets": s.rebuckets,
        "skel_panels": s.skel_panels, "tuned": s.tuned,
        "level_ms": list(s.level_ms[:L]), "top_ms": s.top_ms,
        "precision": s.precision, "retried": bool(s.retried),
    }


def hifde_profile(F: Factor, class_mask: int, level: int = -1):
    """Time the launches of the kernel classes in ``class_mask`` at tree
    level ``level`` (-1: all) with HIP events; 0 stops."""
    check(lib().hifde_profile(F._h, int(class_mask), int(level)))


def hifde_profile_read(F: Factor, cls: int) -> dict:
    """Launches, summed event milliseconds and algorithmic bytes/flops of
    class ``cls`` since the last read."""
    p = Prof()
    check(lib().hifde_profile_read(F._h, int(cls), C.byref(p)))
    return {"launches": p.launches, "ms": p.ms, "bytes": p.bytes, "flops": p.flops}


def hifde_export_sets(F: Factor, level2: int):
    """List of ``(id, [list0, list1, list2, list3])`` with numpy int32 lists."""
    s = Sets()
    check(lib().hifde_export_sets(F._h, level2, C.byref(s)))
    cnt = s.count
    ids = np.zeros(cnt, dtype=np.int64)
    offs = [np.zeros(cnt + 1, dtype=np.int64) for _ in range(4)]
    lists = [np.zeros(max(1, s.total[w]), dtype=np.int32) for w in range(4)]
    s2 = Sets()
    s2.ids = ids.ctypes.data_as(C.POINTER(C.c_int64))
    for w in range(4):
        s2.offs[w] = offs[w].ctypes.data_as(C.POINTER(C.c_int64))
        s2.lists[w] = lists[w].ctypes.data_as(C.POINTER(C.c_int32))
    check(lib().hifde_export_sets(F._h, level2, C.byref(s2)))
    out = []
    for i in range(cnt):
        out.append((int(ids[i]), [lists[w][offs[w][i]:offs[w][i + 1]].copy() for w in range(4)]))
    return out


def hifde_plan_replay(tree: Tree, redundant_level) -> Factor:
    """Host-only replay of the index-set construction with given skeletons
    (``redundant_level[d] = 2l+1`` if unknown d is redundant at level l+1/2)."""
    rl = np.ascontiguousarray(redundant_level, dtype=np.int32)
    h = C.c_void_p()
    check(lib().hifde_plan_replay(tree._h, rl.ctypes.data_as(C.c_void_p), C.byref(h)))
    return Factor(h, tree)


# ---- skeleton-rank predictor -------------------------------------------

def _f32(t, shape=None):
    if not (t.is_cuda and t.is_contiguous() and str(t.dtype) == "torch.float32"):
        raise HifdeError(-1, "expected a contiguous float32 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise HifdeError(-1, f"expected shape {shape}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def hifde_mlp_forward(params, feat, stream=None):
    """Network outputs (log2(1 + k) predictions) for feat (B x 16)."""
    import torch
    B = feat.shape[0]
    out = torch.empty(B, dtype=torch.float32, device=feat.device)
    check(lib().hifde_mlp_forward(_f32(params, (HIFDE_RANK_PARAMS,)), B,
                                  _f32(feat, (B, HIFDE_RANK_FEATURES)), _f32(out),
                                  _stream(stream)))
    return out


def hifde_mlp_grad(params, feat, target, stream=None):
    """(gradient of the mean squared error, loss tensor of one float)."""
    import torch
    B = feat.shape[0]
    nb = C.c_int64()
    check(lib().hifde_mlp_workspace(B, C.byref(nb)))
    work = torch.empty(nb.value // 4, dtype=torch.float32, device=feat.device)
    g = torch.empty(HIFDE_RANK_PARAMS, dtype=torch.float32, device=feat.device)
    loss = torch.empty(1, dtype=torch.float32, device=feat.device)
    check(lib().hifde_mlp_grad(_f32(params, (HIFDE_RANK_PARAMS,)), B,
                               _f32(feat, (B, HIFDE_RANK_FEATURES)), _f32(target, (B,)),
                               _f32(g), _f32(loss), _f32(work), _stream(stream)))
    return g, loss


def hifde_mlp_grad_noalloc(params, feat, target, grad, loss, stream=None):
    """As :func:`hifde_mlp_grad` into the caller's ``grad`` (HIFDE_RANK_PARAMS
    floats) and ``loss`` (one float), with the library's static workspace:
    the call allocates no device memory."""
    B = feat.shape[0]
    check(lib().hifde_mlp_grad_noalloc(_f32(params, (HIFDE_RANK_PARAMS,)), B,
                                       _f32(feat, (B, HIFDE_RANK_FEATURES)), _f32(target, (B,)),
                                       _f32(grad, (HIFDE_RANK_PARAMS,)), _f32(loss, (1,)),
                                       _stream(stream)))


def hifde_mlp_adam(params, grad, m, v, step: int, lr: float, stream=None):
    """One Adam step in place on params (m, v: moment tensors)."""
    check(lib().hifde_mlp_adam(_f32(params), _f32(grad), _f32(m), _f32(v), int(step),
                               float(lr), _stream(stream)))


def hifde_rank_features(F: Factor, level: int, stream=None):
    """(features B x 16, targets log2(1 + k)) of the groups of level + 1/2."""
    import torch
    ng = C.c_int64()
    check(lib().hifde_rank_features(F._h, int(level), None, None, 0, C.byref(ng), None))
    B = ng.value
    feat = torch.zeros((max(B, 1), HIFDE_RANK_FEATURES), dtype=torch.float32, device="cuda")
    tgt = torch.zeros(max(B, 1), dtype=torch.float32, device="cuda")
    if B > 0:
        check(lib().hifde_rank_features(F._h, int(level), _f32(feat), _f32(tgt), B,
                                        C.byref(ng), _stream(stream)))
    return feat[:B], tgt[:B]


def hifde_set_rank_model(tree: Tree, weights):
    """Rank-predictor weights (HIFDE_RANK_PARAMS floats, host) for later
    factorizations of ``tree`` with HIFDE_USE_RANK_MODEL; None removes it."""
    if weights is None:
        check(lib().hifde_set_rank_model(tree._h, None, 0))
        return
    w = np.ascontiguousarray(weights, dtype=np.float32).ravel()
    check(lib().hifde_set_rank_model(tree._h, w.ctypes.data_as(C.c_void_p), w.size))
