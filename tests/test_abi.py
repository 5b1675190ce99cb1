"""The C-ABI library on the CPU: it loads, exports every function that
include/hifde.h declares, rejects invalid trees, and its host planner
reproduces the oracle's tree and index sets bit-exactly when it is given the
oracle's skeleton choices (hifde_plan_replay needs no GPU).

No test here launches device work.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import hifde as OH
from synth import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "hifde.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hifde_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    import paper_1307_2895_amd as H
    lib = H.lib()
    names = _header_functions()
    assert "hifde_factor" in names and "hifde_pcg" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding lists exactly the declared functions
    assert sorted(H._lib.EXPORTED) == names


@pytest.mark.parametrize("dim,n,leaf,skip", [
    (4, 64, 8, 0),     # dim not 2 or 3
    (2, 64, 1, 0),     # leaf < 2
    (2, 8, 8, 0),      # one leaf box per side
    (2, 5, 8, 0),      # n below the leaf size
    (2, 65, 8, 0),     # ceil(n/leaf) = 9 not a power of two
    (2, 64, 8, -1),    # negative skip
    (3, 2048, 8, 0),   # N >= 2^31
])
def test_build_tree_rejects_invalid(dim, n, leaf, skip):
    import paper_1307_2895_amd as H
    with pytest.raises(H.HifdeError) as ei:
        H.hifde_build_tree(dim, n, leaf, skip)
    assert ei.value.code == H.HIFDE_EINVAL
    assert H.lib().hifde_last_error()


def test_null_arguments_are_errors():
    import paper_1307_2895_amd as H
    lib = H.lib()
    assert lib.hifde_build_tree(2, 64, 8, 0, None) == H.HIFDE_EINVAL
    assert lib.hifde_stats(None, None) == H.HIFDE_EINVAL
    assert lib.hifde_profile(None, 1, -1) == H.HIFDE_EINVAL
    assert lib.hifde_plan_replay(None, None, None) == H.HIFDE_EINVAL


def _redundant_levels(OF):
    red = np.full(OF.N, -1, dtype=np.int32)
    for l, lev in enumerate(OF.levels):
        for g in lev.groups:
            red[np.asarray(g.rd, dtype=np.int64)] = 2 * l + 1
    return red


def _compare_replay(OF, P):
    import paper_1307_2895_amd as H
    sets, top = OH.export_sets(OF)
    for l, lev in enumerate(sets):
        gc = H.hifde_export_sets(P, 2 * l)
        assert len(gc) == len(lev["cells"]), f"cell count at level {l}"
        for (cid, p, q), (hid, hl) in zip(lev["cells"], gc):
            assert cid == hid
            assert np.array_equal(p, hl[0]), f"p of cell {cid}, level {l}"
            assert np.array_equal(q, hl[1]), f"front of cell {cid}, level {l}"
        gg = H.hifde_export_sets(P, 2 * l + 1)
        assert len(gg) == len(lev["groups"]), f"group count at level {l}+1/2"
        for (gid, c, cN, sk, rd), (hid, hl) in zip(lev["groups"], gg):
            assert gid == hid
            assert np.array_equal(c, hl[0]), f"c of group {gid}, level {l}+1/2"
            assert np.array_equal(cN, hl[1]), f"c^N of group {gid}, level {l}+1/2"
            assert np.array_equal(sk, hl[2]) and np.array_equal(rd, hl[3])
    tp = H.hifde_export_sets(P, 2 * OF.L)
    assert np.array_equal(tp[0][1][0], top)


REPLAY_CASES = [
    # dim, n, leaf, eps, field, seed, skip
    (2, 64, 8, 1e-6, "const", None, 0),
    (2, 64, 8, 1e-6, "bernoulli_contrast", 2, 0),
    (2, 48, 3, 1e-6, "loguniform", 7, 0),
    (2, 64, 4, 1e-3, "loguniform", 3, 1),
    (2, 32, 4, 0.0, "const", None, 0),
    (3, 16, 4, 1e-6, "const", None, 0),
    (3, 16, 2, 1e-3, "lognormal_grf", 4, 0),
    # ragged grids: the last box along each axis is short
    (2, 60, 8, 1e-6, "loguniform", 7, 0),
    (2, 57, 8, 1e-3, "bernoulli_contrast", 2, 0),   # last leaf box one wide
    (3, 30, 4, 1e-6, "const", None, 0),
]


@pytest.mark.parametrize("dim,n,m,eps,field,seed,skip", REPLAY_CASES)
def test_plan_replay_matches_oracle(dim, n, m, eps, field, seed, skip):
    import paper_1307_2895_amd as H
    a = W.make_field(dim, n, field, seed)
    OF = OH.factor(dim, n, m, a, eps=eps, skip_levels=skip)
    T = H.hifde_build_tree(dim, n, m, skip)
    P = H.hifde_plan_replay(T, _redundant_levels(OF))
    _compare_replay(OF, P)
    st = H.hifde_stats(P)
    assert st["N"] == n ** dim and st["levels"] == OF.L
    assert st["top_size"] == len(OH.export_sets(OF)[1])


def test_plan_replay_threads_agree(monkeypatch):
    """The planner's worker threads do not change any index set."""
    import subprocess
    import sys
    code = (
        "import sys, numpy as np; sys.path.insert(0, %r); sys.path.insert(0, %r);"
        "import paper_1307_2895_amd as H; from synth import workloads as W;"
        "from oracle import hifde as OH;"
        "a = W.make_field(2, 64, 'loguniform', 9);"
        "OF = OH.factor(2, 64, 4, a, eps=1e-4);"
        "red = np.full(OF.N, -1, dtype=np.int32)\n"
        "for l, lev in enumerate(OF.levels):\n"
        "    for g in lev.groups: red[np.asarray(g.rd, dtype=np.int64)] = 2*l+1\n"
        "P = H.hifde_plan_replay(H.hifde_build_tree(2, 64, 4, 0), red)\n"
        "out = []\n"
        "for l2 in range(2*OF.L+1):\n"
        "    for gid, ls in H.hifde_export_sets(P, l2): out.append((gid, [x.tolist() for x in ls]))\n"
        "print(hash(repr(out)))\n"
    ) % (ROOT, os.path.join(ROOT, "tests"))
    res = []
    for t in ("1", "5"):
        env = dict(os.environ, HIFDE_PLAN_THREADS=t, PYTHONHASHSEED="0")
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=300)
        assert r.returncode == 0, r.stderr
        res.append(r.stdout.strip())
    assert res[0] == res[1]


def test_plan_replay_rejects_null_tree():
    import paper_1307_2895_amd as H
    out = C.c_void_p()
    rc = H.lib().hifde_plan_replay(None, None, C.byref(out))
    assert rc == H.HIFDE_EINVAL


@pytest.mark.parametrize("dim,n,m,eps,field,seed,skip", REPLAY_CASES)
def test_plan_replay_flop_count_matches_oracle(dim, n, m, eps, field, seed, skip):
    """The library's algorithmic flop count (reported by hifde_stats and used
    for every factorization rate) equals the oracle's factor_flops when both
    hold the same index sets."""
    import paper_1307_2895_amd as H
    a = W.make_field(dim, n, field, seed)
    OF = OH.factor(dim, n, m, a, eps=eps, skip_levels=skip)
    T = H.hifde_build_tree(dim, n, m, skip)
    P = H.hifde_plan_replay(T, _redundant_levels(OF))
    st = H.hifde_stats(P)
    assert st["factor_flops"] == pytest.approx(OH.factor_flops(OF), rel=1e-12)
