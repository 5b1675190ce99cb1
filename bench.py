"""Throughput of the HIF-DE hot path on one MI355X.

One step = one pass of the whole path over one batch of synthetic input:
hifde_factor (stencil assembly, every level's batched elimination and
skeletonization, the FP64 top block) followed by hifde_pcg (FP64 conjugate
gradients preconditioned by F^-1) on all right-hand sides to a relative
residual of 1e-12.  Inputs (coefficients and right-hand sides) are resident
in HBM before the timed region starts.

Prints one JSON line.  ``value`` is the whole-step throughput
N * nrhs / (t_factor + t_pcg) in DOF*RHS/s; the factor DOF/s and solve
DOF*RHS/s components, the plain FP64 path, the roofline of the dominant
kernel and the CPU oracle baseline are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="contrast2d_n1024")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 GPU path")
    ap.add_argument("--cpu-n", type=int, default=256, help="grid side of the CPU oracle sample")
    return ap.parse_args()


def cpu_baseline(w, n_sample, nrhs):
    """The oracle, untouched, on a bounded sample of the same workload recipe:
    same field recipe, leaf, eps and right-hand-side distribution on an
    n_sample^dim grid; factor + PCG (FP64, tol 1e-12) on nrhs columns."""
    from oracle import hifde as OH
    from oracle import pcg as OP
    from synth import workloads as W
    a = W.make_field(w.dim, n_sample, w.field, w.seed_a)
    f = W.make_rhs(n_sample ** w.dim, nrhs, w.seed_f)
    t0 = time.perf_counter()
    F = OH.factor(w.dim, n_sample, w.leaf, a, eps=w.eps)
    t1 = time.perf_counter()
    _, its, rr = OP.pcg_multi(F.A, f, lambda r: OH.solve(F, r), 1e-12, 200)
    t2 = time.perf_counter()
    Ns = n_sample ** w.dim
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": Ns * nrhs / (t2 - t0),
        "unit": "DOF*RHS/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{w.field} field, {w.dim}D n={n_sample} (N={Ns}), leaf {w.leaf}, eps {w.eps}, "
                   f"{nrhs} RHS; FP64 factor {t1 - t0:.2f} s + PCG to 1e-12 {t2 - t1:.2f} s "
                   f"(iters {int(np.max(its))})"),
        "factor_dof_per_s": Ns / (t1 - t0),
        "solve_dof_rhs_per_s": Ns * nrhs / (t2 - t1),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); "
              "the method's multi-GPU sharding is described in DESIGN.md and not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1307_2895_amd as H
    from synth import workloads as W

    w = W.workload(args.workload)
    N, nrhs = w.N, w.nrhs
    a_h = W.make_coefficients(w)
    f_h = W.make_rhs(N, nrhs, w.seed_f)
    dev = torch.device("cuda:0")
    a_d = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in a_h]
    f_d = torch.from_numpy(f_h).to(dev)
    tree = H.hifde_build_tree(w.dim, w.n, w.leaf, 0)
    prec = H.HIFDE_MIXED if w.precision == "mixed" else H.HIFDE_FP64

    def step(p):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = H.hifde_factor(tree, a_d, None, w.eps, p)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        u, its, rel = H.hifde_pcg(F, f_d, tol=1e-12, maxit=200)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        st = H.hifde_stats(F)
        F.free()
        return t1 - t0, t2 - t1, its, rel, st

    for _ in range(args.warmup):
        step(prec)
        print("warmup step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tf, tp, iters = [], [], None
    t_begin = time.perf_counter()
    for k in range(args.steps):
        a, b, its, rel, st = step(prec)
        tf.append(a)
        tp.append(b)
        iters, relres, stats = its, rel, st
        print(f"step {k}: factor {a*1e3:.1f} ms, pcg {b*1e3:.1f} ms, iters {int(its.max())}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_begin
    ms_step = 1e3 * t_total / args.steps
    t_f, t_p = float(np.median(tf)), float(np.median(tp))

    out = {
        "metric": "factor DOF/s + solve DOF*RHS/s, mixed vs FP64 GPU path at 1e-12 PCG residual",
        "value": N * nrhs / (t_total / args.steps),
        "unit": "DOF*RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 factor/F^-1, f64 PCG" if prec == H.HIFDE_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "dim": w.dim, "n": w.n, "N": N, "leaf": w.leaf,
                   "eps": w.eps, "field": w.field, "nrhs": nrhs, "tol": 1e-12},
        "components": {
            "factor_dof_per_s": N / t_f,
            "solve_dof_rhs_per_s": N * nrhs / t_p,
            "factor_ms": 1e3 * t_f,
            "pcg_ms": 1e3 * t_p,
            "pcg_iters_max": int(np.max(iters)),
            "pcg_relres_max": float(np.max(relres)),
            "top_size": stats["top_size"],
            "factor_bytes": stats["factor_bytes"],
            "factor_gflop": stats["factor_flops"] / 1e9,
        },
    }
    if not args.no_fp64 and prec == H.HIFDE_MIXED:
        a, b, its, rel, st = step(H.HIFDE_FP64)
        out["fp64_path"] = {
            "factor_dof_per_s": N / a, "solve_dof_rhs_per_s": N * nrhs / b,
            "factor_ms": 1e3 * a, "pcg_ms": 1e3 * b, "pcg_iters_max": int(np.max(its)),
            "step_dof_rhs_per_s": N * nrhs / (a + b),
        }
        out["speedup_mixed_vs_fp64"] = (a + b) / (t_f + t_p)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_n, nrhs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
