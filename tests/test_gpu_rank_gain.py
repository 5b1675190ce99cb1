"""GPU: what the trained rank predictor gains, and that it never changes the
factorization.

Three ways to launch each level's skeleton-front eliminations are compared
on held-out problems of the rank-model workload's field recipe:
  * after the IDs' ranks reach the host (the method without the predictor),
  * before, bounded by the predicted ranks (HIFDE_USE_RANK_MODEL),
  * before, bounded by the worst case k = 0 (HIFDE_PRESIZE_WORST_CASE),
plus an adversarial model whose every prediction is wrong.  Skeleton sets
and (in FP64) F^-1 f must be bitwise identical in all four; the predictor
must launch no more panel sweeps than the worst case, and a misprediction
must show up as a re-launch (rebucket), never as a different result.
"""
import time

import numpy as np
import pytest

from oracle import mlp as M
from synth import workloads as W

from _helpers import torch_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _features(problems, prec=0):
    import paper_1307_2895_amd as H
    fs, ts = [], []
    for n, seed in problems:
        a = W.make_field(2, n, "loguniform", seed)
        T = H.hifde_build_tree(2, n, 16, 0)
        F = H.hifde_factor(T, torch_inputs(a), None, 1e-6, prec)
        for level in range(H.hifde_stats(F)["levels"]):
            f, t = H.hifde_rank_features(F, level)
            fs.append(f)
            ts.append(t)
    return torch.cat(fs), torch.cat(ts)


def _train(X, t, steps=1500, lr=3e-3):
    import paper_1307_2895_amd as H
    theta = torch.from_numpy(M.init_params(16, 64, seed=0).astype(np.float32)).cuda()
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    for step in range(1, steps + 1):
        g, _ = H.hifde_mlp_grad(theta, X, t)
        H.hifde_mlp_adam(theta, g, m, v, step, lr)
    return theta.cpu().numpy()


def _sets(F, L):
    import paper_1307_2895_amd as H
    out = []
    for l2 in range(2 * L + 1):
        out.append([(gid, [x.tolist() for x in ls]) for gid, ls in H.hifde_export_sets(F, l2)])
    return out


@pytest.fixture(scope="module")
def trained():
    X, t = _features([(128, 500), (128, 501), (256, 502), (256, 503)])
    return _train(X, t)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,seed", [(256, 512), (512, 513)])
def test_predictor_changes_nothing_and_bounds_launches(trained, prec, n, seed):
    import paper_1307_2895_amd as H
    a = W.make_field(2, n, "loguniform", seed)
    T = H.hifde_build_tree(2, n, 16, 0)
    f = torch.from_numpy(W.make_rhs(n * n, 4, 9)).cuda()
    adversarial = np.zeros(H.HIFDE_RANK_PARAMS, dtype=np.float32)
    adversarial[-1] = 20.0          # log2(1 + k) = 20: every group predicted whole
    runs = {}
    for name, flags, model in [("sync", 0, None), ("model", H.HIFDE_USE_RANK_MODEL, trained),
                               ("worst", H.HIFDE_PRESIZE_WORST_CASE, None),
                               ("adversarial", H.HIFDE_USE_RANK_MODEL, adversarial)]:
        H.hifde_set_rank_model(T, model)
        H.hifde_factor(T, torch_inputs(a), None, 1e-6, prec, flags=flags).free()   # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = H.hifde_factor(T, torch_inputs(a), None, 1e-6, prec, flags=flags)
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        st = H.hifde_stats(F)
        u = H.hifde_solve(F, f)
        runs[name] = (F, st, u, tf)
        print(f"n={n} prec={prec} {name:12s} t_factor {tf * 1e3:7.2f} ms  rank MAE "
              f"{st['rank_mae']:.3f} over {st['rank_groups']} groups  rebuckets "
              f"{st['rebuckets']}  skeleton panel sweeps {st['skel_panels']}")
    L = runs["sync"][1]["levels"]
    ref_sets = _sets(runs["sync"][0], L)
    for name in ("model", "worst", "adversarial"):
        assert _sets(runs[name][0], L) == ref_sets, name
        if prec == 0:
            assert torch.equal(runs[name][2], runs["sync"][2]), name
        else:
            du = (runs[name][2] - runs["sync"][2]).abs().max().item()
            assert du <= 1e-4 * runs["sync"][2].abs().max().item(), name
    assert runs["model"][1]["skel_panels"] <= runs["worst"][1]["skel_panels"]
    assert runs["adversarial"][1]["rebuckets"] >= 1
    assert runs["model"][1]["rank_groups"] == sum(len(s) for s in ref_sets[1::2][:L])
    H.hifde_set_rank_model(T, None)


def test_model_flag_requires_a_model():
    import paper_1307_2895_amd as H
    a = W.make_field(2, 64, "loguniform", 1)
    T = H.hifde_build_tree(2, 64, 8, 0)
    with pytest.raises(H.HifdeError) as ei:
        H.hifde_factor(T, torch_inputs(a), None, 1e-6, 0, flags=H.HIFDE_USE_RANK_MODEL)
    assert ei.value.code == H.HIFDE_ESTATE
