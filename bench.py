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

# The kernel the roofline object describes: the upward sweep of F^-1 over
# the level-0 cells, both colors in one launch (k_sweep_up_c<float, float,
# 1, true>, the 16-right-hand-side instance), the kernel with the most time
# per step.  Its launches are exactly those of the profile class
# HIFDE_PROF_SWEEP_UP_ONE.
DOMINANT_KERNEL = "k_sweep_up_c<float, float, 1, true>"
DOMINANT_SOURCE = os.path.join(ROOT, "paper_1307_2895_amd", "csrc", "kernels_solve.inc")
CALIB_COPY_BYTES = 512 << 20


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="contrast2d_n1024")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 GPU path")
    ap.add_argument("--cpu-n", type=int, default=256, help="grid side of the CPU oracle sample")
    ap.add_argument("--calib-copy", action="store_true",
                    help=f"first run one plain device copy of {CALIB_COPY_BYTES >> 20} MiB "
                         "(scale reference for HBM counters)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarize two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of "
                         "this script with --calib-copy and exit")
    return ap.parse_args()


def source_sha(path):
    import hashlib
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def traffic_file(workload):
    name = DOMINANT_KERNEL.split("<")[0]
    return os.path.join(ROOT, "profiles", f"traffic_{name}_{workload}.txt")


def read_traffic(workload):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when absent or taken on a different kernel source."""
    path = traffic_file(workload)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != source_sha(DOMINANT_SOURCE):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _pmc_rows(d, counter):
    """(kernel name, grid size, value) rows of a rocprofv3 counter CSV."""
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") == counter:
                    rows.append((r["Kernel_Name"], int(r.get("Grid_Size", 0) or 0),
                                 float(r["Counter_Value"])))
    return rows


def pmc_summary(fetch_dir, write_dir, workload):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the dominant kernel,
    scaled by what the same counters read for the calibration copy."""
    out = {}
    for key, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = _pmc_rows(d, counter)
        # per dispatch: the counter is reported per dispatch (summed over instances)
        wide = [v for n, g, v in rows if "copybuffer" in n.lower()]
        narrow = [v for n, g, v in rows if "MulFunctor" in n]
        dom = [v for n, g, v in rows if DOMINANT_KERNEL.replace(" ", "") in n.replace(" ", "")]
        if not wide or not narrow or not dom:
            raise SystemExit(f"{counter}: calibration copies or {DOMINANT_KERNEL} not found in {d}")
        kib = CALIB_COPY_BYTES / 1024.0
        out[key] = (len(dom), float(np.mean(dom)), kib / max(narrow), kib / max(wide))
    nd, fkib, fs, fs_w = out["fetch"]
    _, wkib, ws, ws_w = out["write"]
    traffic = (fkib * fs + wkib * ws) * 1024.0
    lines = [
        f"# HBM traffic of {DOMINANT_KERNEL} on {workload} from rocprofv3 counters",
        "# commands (from the repository root, TMPDIR=/tmp); the scales divide the known",
        "# size of a 4-byte-per-lane elementwise copy by what the counter reads for it",
        f"#   rocprofv3 --pmc FETCH_SIZE -f csv -d <FETCH_DIR> -- python bench.py --steps 1 "
        f"--warmup 0 --no-cpu --no-fp64 --calib-copy",
        f"#   rocprofv3 --pmc WRITE_SIZE -f csv -d <WRITE_DIR> -- python bench.py --steps 1 "
        f"--warmup 0 --no-cpu --no-fp64 --calib-copy",
        f"#   python bench.py --pmc-summary <FETCH_DIR> <WRITE_DIR>",
        f"kernel: {DOMINANT_KERNEL}",
        f"kernel_source_sha256: {source_sha(DOMINANT_SOURCE)}",
        f"dispatches: {nd}",
        f"fetch_kib_per_dispatch: {fkib:.1f}",
        f"write_kib_per_dispatch: {wkib:.1f}",
        f"copy_fetch_scale: {fs:.4f}",
        f"copy_write_scale: {ws:.4f}",
        f"# the same counters on the runtime's block copy (wide loads) give scales "
        f"{fs_w:.4f} (fetch) and {ws_w:.4f} (write)",
        f"traffic_bytes_per_launch_wide_scale: {(fkib * fs_w + wkib * ws_w) * 1024.0:.0f}",
        f"traffic_bytes_per_launch: {traffic:.0f}",
    ]
    return "\n".join(lines)


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
    if args.pmc_summary:
        print(pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.workload))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): "
              "the path runs on one GPU; sharding it over several is not built.",
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

    if args.calib_copy:
        # two plain copies of known size: a runtime block copy (wide loads)
        # and an elementwise scale by 1 on 4-byte-misaligned views, which
        # runs with one 4-byte load and store per lane like the sweep kernels
        src = torch.ones(CALIB_COPY_BYTES // 4 + 1, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst[:-1].copy_(src[:-1])
        torch.mul(src[1:], 1.0, out=dst[1:])
        torch.cuda.synchronize()
        del src, dst

    prof = {"launches": 0, "ms": 0.0, "bytes": 0.0, "flops": 0.0}

    def step(p, profile=False, tune=False):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = H.hifde_factor(tree, a_d, None, w.eps, p, flags=H.HIFDE_AUTOTUNE if tune else 0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if profile:
            H.hifde_profile(F, 1 << H.HIFDE_PROF_SWEEP_UP_ONE, -1)
        u, its, rel = H.hifde_pcg(F, f_d, tol=1e-12, maxit=200)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if profile:
            r = H.hifde_profile_read(F, H.HIFDE_PROF_SWEEP_UP_ONE)
            for k in prof:
                prof[k] += r[k]
        st = H.hifde_stats(F)
        F.free()
        return t1 - t0, t2 - t1, its, rel, st

    # warmup: the first step autotunes the launch variants of every size
    # bucket; the tree keeps the choices for the timed steps
    for i in range(args.warmup):
        step(prec, tune=(i == 0))
        print("warmup step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tf, tp, iters = [], [], None
    t_begin = time.perf_counter()
    for k in range(args.steps):
        a, b, its, rel, st = step(prec, profile=True)
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
    nl = max(1, prof["launches"])
    avg_s = prof["ms"] / nl / 1e3
    bytes_launch = prof["bytes"] / nl
    achieved = bytes_launch / avg_s / 1e9 if avg_s > 0 else 0.0
    traffic = read_traffic(w.name)
    out["roofline"] = {
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
        "kernel": DOMINANT_KERNEL, "launches": prof["launches"],
        "avg_launch_us": avg_s * 1e6, "algorithmic_bytes_per_launch": bytes_launch,
        "mfma_tflops": prof["flops"] / nl / avg_s / 1e12 if avg_s > 0 else 0.0,
    }
    if not args.no_fp64 and prec == H.HIFDE_MIXED:
        step(H.HIFDE_FP64, tune=True)        # tune the FP64 buckets (untimed)
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
