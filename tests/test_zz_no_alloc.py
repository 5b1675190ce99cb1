"""hifde_mlp_grad_noalloc (the rank predictor's gradient with the library's
static device workspace) against hifde_mlp_grad (caller's workspace): the
same kernels in the same order, so the gradients and losses agree bit for
bit.  Two calls in a row, the second with fewer samples, show that the
static array's leftover contents from a larger call do not leak into a
smaller one."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _inputs(B, seed):
    import paper_1307_2895_amd as H
    g = np.random.Generator(np.random.PCG64(seed))
    params = torch.from_numpy(
        (0.2 * g.standard_normal(H.HIFDE_RANK_PARAMS)).astype(np.float32)).cuda()
    feat = torch.from_numpy(
        g.standard_normal((B, H.HIFDE_RANK_FEATURES)).astype(np.float32)).cuda()
    target = torch.from_numpy((3.0 * g.random(B)).astype(np.float32)).cuda()
    return params, feat, target


def test_noalloc_grad_matches_workspace_grad_twice():
    import paper_1307_2895_amd as H
    grad = torch.empty(H.HIFDE_RANK_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    for B, seed in ((3000, 71), (700, 72)):
        print(f"case nbatch={B} seed={seed}", flush=True)
        params, feat, target = _inputs(B, seed)
        g_ref, l_ref = H.hifde_mlp_grad(params, feat, target)
        grad.fill_(float("nan"))
        loss.fill_(float("nan"))
        H.hifde_mlp_grad_noalloc(params, feat, target, grad, loss)
        torch.cuda.synchronize()
        assert torch.isfinite(g_ref).all() and torch.isfinite(l_ref).all()
        assert torch.equal(grad, g_ref), float((grad - g_ref).abs().max())
        assert torch.equal(loss, l_ref), (float(loss), float(l_ref))


def test_noalloc_grad_rejects_oversized_batch():
    import paper_1307_2895_amd as H
    lib = H.lib()
    B = H.HIFDE_MLP_NOALLOC_MAX_BATCH + 1
    # rejected on the host before any device work: the pointers are never used
    dummy = C.c_void_p(256)
    rc = lib.hifde_mlp_grad_noalloc(dummy, B, dummy, dummy, dummy, dummy, None)
    assert rc == H.HIFDE_EINVAL
    assert b"HIFDE_MLP_NOALLOC_MAX_BATCH" in lib.hifde_last_error()
    rc = lib.hifde_mlp_grad_noalloc(None, 16, dummy, dummy, dummy, dummy, None)
    assert rc == H.HIFDE_EINVAL
