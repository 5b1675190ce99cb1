"""Accuracy of the mixed-precision preconditioner (FP32 cells, groups, IDs
and sweeps; FP64 top block) against the FP64 oracle at the same eps.

Reported per case: the one-application relative residual
||A F^-1 f - f|| / ||f|| of both, their ratio, e_s = ||I - A F^-1|| (power
iteration, Section 5) of both, and the PCG iteration counts.

Bars.  The FP64 GPU path: within 2x of the oracle at the same eps.  The
mixed paths (HIFDE_MIXED, and HIFDE_MIXED_ELIM64 whose cell eliminations are
double) round every cell or group and ID step to float (unit roundoff
u = 6e-8); with the growth of the ID's triangular solve and of the Schur
updates on these grids (about 100-200) that acts as a tolerance of about
1e-5, so its one-application residual must stay within 2x of the oracle's
at EPS_EFF = max(eps, 1e-5).  Its PCG must reach 1e-12 with a solution
within 1e-10 of the oracle's (||A (u - u_oracle)|| / ||f||)."""
import numpy as np
import pytest

from oracle import errest as OE
from oracle import hifde as OH
from oracle import pcg as OP
from synth import workloads as W

from _helpers import gpu_factor, oracle_factor, rel_residual

pytestmark = pytest.mark.gpu

EPS32_FLOOR = 1e-5

torch = pytest.importorskip("torch")

CASES = [
    # dim, n, leaf, eps, field, seed
    (2, 64, 8, 1e-6, "const", None),
    (2, 64, 8, 1e-6, "bernoulli_contrast", 2),
    (2, 256, 16, 1e-6, "bernoulli_contrast", 2),
    (3, 16, 4, 1e-6, "const", None),
    (3, 32, 4, 1e-6, "const", None),
]


def _solver(F):
    import paper_1307_2895_amd as H

    def s(v):
        v2 = np.ascontiguousarray(v.reshape(v.shape[0], -1))
        u = H.hifde_solve(F, torch.from_numpy(v2).cuda()).cpu().numpy()
        return u.reshape(v.shape)
    return s


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("dim,n,m,eps,field,seed", CASES)
def test_mixed_one_application_residual(dim, n, m, eps, field, seed, prec):
    import paper_1307_2895_amd as H
    print(f"case dim={dim} n={n} leaf={m} eps={eps} field={field} prec={prec}", flush=True)
    a = W.make_field(dim, n, field, seed)
    OF = oracle_factor(dim, n, m, a, eps)
    N = n ** dim
    f = W.make_rhs(N, 4, 11)
    _, Fm = gpu_factor(dim, n, m, a, eps, prec)
    _, Fd = gpu_factor(dim, n, m, a, eps, 0)
    rm = rel_residual(OF.A, _solver(Fm)(f), f)
    rd = rel_residual(OF.A, _solver(Fd)(f), f)
    ro = rel_residual(OF.A, OH.solve(OF, f), f)
    es_m = OE.e_s(OF.A, _solver(Fm), seed=1)
    es_o = OE.e_s(OF.A, lambda v: OH.solve(OF, v), seed=1)
    ug, its, rel = H.hifde_pcg(Fm, torch.from_numpy(f).cuda(), tol=1e-12, maxit=200)
    _, ito, _ = OP.pcg_multi(OF.A, f, lambda r: OH.solve(OF, r), 1e-12, 200)
    eps_eff = max(eps, EPS32_FLOOR)
    OFe = OF if eps_eff == eps else oracle_factor(dim, n, m, a, eps_eff)
    re = ro if eps_eff == eps else rel_residual(OFe.A, OH.solve(OFe, f), f)
    print(f"residual mixed {rm.max():.3e} fp64-gpu {rd.max():.3e} oracle {ro.max():.3e} "
          f"(at {eps_eff:g}: {re.max():.3e}) ratio mixed/oracle {np.max(rm / ro):.3f} "
          f"(at {eps_eff:g}: {np.max(rm / re):.3f}); e_s mixed {es_m:.3e} oracle {es_o:.3e}; "
          f"pcg iters mixed {its.tolist()} oracle {ito.tolist()}", flush=True)
    assert np.all(rd <= 2.0 * ro)
    assert np.all(rm <= 2.0 * re)
    assert np.all(rel <= 1.5e-12), rel
    uo, _, _ = OP.pcg_multi(OF.A, f, lambda r: OH.solve(OF, r), 1e-12, 200)
    d = np.linalg.norm(OF.A @ (ug.cpu().numpy() - uo), axis=0) / np.linalg.norm(f, axis=0)
    assert np.all(d <= 1e-10), d
