"""GPU: the captured (HIP graph) application of F^-1 against direct
launches, and the determinism check of the factorization.

The sweeps are deterministic (no atomics, fixed reduction orders), so a
replayed graph must reproduce the direct launches bit for bit; every replay
is checked, with eager work and synchronizations between replays.
"""
import numpy as np
import pytest

from synth import workloads as W

from _helpers import torch_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("nrhs", [1, 16, 40])
def test_graph_replays_match_direct_launches(prec, nrhs):
    import paper_1307_2895_amd as H
    print(f"case prec={prec} nrhs={nrhs}", flush=True)
    dim, n, m = 2, 64, 8
    a = W.make_field(dim, n, "bernoulli_contrast", 3)
    T = H.hifde_build_tree(dim, n, m, 0)
    Fg = H.hifde_factor(T, torch_inputs(a), None, 1e-6, prec)
    Fd = H.hifde_factor(T, torch_inputs(a), None, 1e-6, prec, flags=H.HIFDE_NO_GRAPH)
    f = torch.from_numpy(W.make_rhs(n ** dim, nrhs, 5)).cuda()
    ud = H.hifde_solve(Fd, f)
    torch.cuda.synchronize()
    for rep in range(4):
        ug = H.hifde_solve(Fg, f)
        torch.cuda.synchronize()
        assert torch.equal(ug, ud), f"replay {rep} differs"
        # eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
    # a different right-hand-side count recaptures
    f2 = f[:, :1].contiguous()
    assert torch.equal(H.hifde_solve(Fg, f2), H.hifde_solve(Fd, f2))


def test_graph_pcg_matches_direct():
    import paper_1307_2895_amd as H
    dim, n, m = 2, 64, 8
    a = W.make_field(dim, n, "loguniform", 4)
    T = H.hifde_build_tree(dim, n, m, 0)
    Fg = H.hifde_factor(T, torch_inputs(a), None, 1e-6, H.HIFDE_MIXED)
    Fd = H.hifde_factor(T, torch_inputs(a), None, 1e-6, H.HIFDE_MIXED, flags=H.HIFDE_NO_GRAPH)
    f = torch.from_numpy(W.make_rhs(n ** dim, 8, 6)).cuda()
    ug, itg, rg = H.hifde_pcg(Fg, f, tol=1e-12)
    ud, itd, rd = H.hifde_pcg(Fd, f, tol=1e-12)
    assert np.array_equal(itg, itd)
    assert torch.equal(ug, ud)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_debug_determinism_flag(prec):
    import paper_1307_2895_amd as H
    dim, n, m = 3, 16, 4
    a = W.make_field(dim, n, "lognormal_grf", 4)
    T = H.hifde_build_tree(dim, n, m, 0)
    F = H.hifde_factor(T, torch_inputs(a), None, 1e-4, prec, flags=H.HIFDE_DEBUG_DETERMINISM)
    assert H.hifde_stats(F)["top_size"] > 0


def test_unknown_flags_rejected():
    import paper_1307_2895_amd as H
    a = W.make_field(2, 32, "const", None)
    T = H.hifde_build_tree(2, 32, 4, 0)
    with pytest.raises(H.HifdeError) as ei:
        H.hifde_factor(T, torch_inputs(a), None, 1e-6, 0, flags=1 << 20)
    assert ei.value.code == H.HIFDE_EINVAL


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("nrhs", [1, 16, 40])
def test_whole_front_sweeps_match_row_tiles(prec, nrhs):
    """The whole-front sweeps (one work-group per front, interpolation fused
    into the skeleton fronts' launches) take the same products in the same
    order as the row-tile forms with separate interpolation launches, so
    F^-1 f must agree bit for bit.  n = 512, leaf 8: 2048 cells per color,
    enough for the whole-front cell launches."""
    import paper_1307_2895_amd as H
    print(f"case prec={prec} nrhs={nrhs}", flush=True)
    dim, n, m = 2, 512, 8
    a = W.make_field(dim, n, "bernoulli_contrast", 7)
    T = H.hifde_build_tree(dim, n, m, 0)
    Fw = H.hifde_factor(T, torch_inputs(a), None, 1e-6, prec)
    Fr = H.hifde_factor(T, torch_inputs(a), None, 1e-6, prec, flags=H.HIFDE_SWEEP_ROW_TILES)
    f = torch.from_numpy(W.make_rhs(n ** dim, nrhs, 8)).cuda()
    uw = H.hifde_solve(Fw, f)
    ur = H.hifde_solve(Fr, f)
    torch.cuda.synchronize()
    assert torch.isfinite(uw).all()
    assert torch.equal(uw, ur)


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("what", ["a_negative", "a_nan", "b_inf"])
def test_invalid_coefficients_rejected(prec, what):
    """Invalid coefficients are reported as HIFDE_EINVAL; the flags k_stencil
    sets are read at the factorization's first synchronization, after the
    level-0 kernels have run on the values (they index by structure only)."""
    import paper_1307_2895_amd as H
    print(f"case prec={prec} {what}", flush=True)
    dim, n, m = 2, 64, 8
    a = W.make_field(dim, n, "loguniform", 11)
    b = None
    if what == "a_negative":
        a[0].flat[5] = -1.0
    elif what == "a_nan":
        a[1].flat[7] = np.nan
    T = H.hifde_build_tree(dim, n, m, 0)
    args = torch_inputs(a)
    if what == "b_inf":
        bb = np.zeros(n ** dim)
        bb[3] = np.inf
        b = torch.from_numpy(bb).cuda()
    with pytest.raises(H.HifdeError) as ei:
        H.hifde_factor(T, args, b, 1e-6, prec)
    assert ei.value.code == H.HIFDE_EINVAL
    # the tree stays usable
    F = H.hifde_factor(T, torch_inputs(W.make_field(dim, n, "loguniform", 11)), None, 1e-6, prec)
    assert H.hifde_stats(F)["top_size"] > 0


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_timed_first_sweep_with_graph_matches_unprofiled(prec):
    """Timing only the one-launch level-0 upward sweep runs that kernel
    directly and the rest of each F^-1 application from a graph captured
    without it; PCG must reproduce the unprofiled run bit for bit, and the
    class must have timed one launch per application."""
    import paper_1307_2895_amd as H
    print(f"case prec={prec}", flush=True)
    dim, n, m, nrhs = 2, 512, 8, 16
    a = W.make_field(dim, n, "bernoulli_contrast", 7)
    T = H.hifde_build_tree(dim, n, m, 0)
    f = torch.from_numpy(W.make_rhs(n ** dim, nrhs, 9)).cuda()
    Fn = H.hifde_factor(T, torch_inputs(a), None, 1e-6, prec)
    un, itn, _ = H.hifde_pcg(Fn, f, tol=1e-10)
    Fp = H.hifde_factor(T, torch_inputs(a), None, 1e-6, prec)
    H.hifde_profile(Fp, 1 << H.HIFDE_PROF_SWEEP_UP_ONE, -1)
    up, itp, _ = H.hifde_pcg(Fp, f, tol=1e-10)
    r = H.hifde_profile_read(Fp, H.HIFDE_PROF_SWEEP_UP_ONE)
    torch.cuda.synchronize()
    assert np.array_equal(itn, itp)
    assert torch.equal(un, up)
    assert r["launches"] == int(np.max(itp))   # one application before each iteration but the last
    assert r["ms"] > 0 and r["bytes"] > 0
