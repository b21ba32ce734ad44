"""Benchmark: heterogeneous-FMM matvecs per second on one MI355X.

Workload: three layers (interfaces y = 0.5 and y = 0; k = 2pi*(80, 120, 100)
top to bottom), N = 10^6 points on 64 random ellipses in the top layer, one
complex128 right-hand side, FP64, tolerance 1e-8, leaf size 64 (seeded
synthetic inputs, see workloads.three_layer_ellipses).

A step is one hfmm_apply (u = A q) with q and u resident in device memory;
the plan (tree, lists, tables) is built before the timed region. Prints one
JSON line. With --gpus other than 1 it exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H-FMM matvecs/sec at N=1e6, 3 layers, rel err 1e-8 (FP64) vs mixed; adjoint s"
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector (and FP64 matrix) peak
PEAK_HBM_GBS = 8000.0


def cpu_baseline_sample(w, seconds_budget=20.0):
    """The oracle on a bounded sample of the same matvec, extrapolated to one full matvec.

    Free part: a few complete target rows (all N sources). Scattered part: the
    per-node source sums over a slice of the sources and the per-node target
    evaluation for a few targets, each scaled to N.
    """
    import numpy as np

    import oracle
    from oracle import sommerfeld as som
    media = oracle.Media(w.k, w.interfaces)
    x = w.xy[:, 0]
    y = media.to_frame(w.xy[:, 1])
    n = w.n
    workers = som._workers()
    rows = 16
    tid = np.arange(0, n, n // rows)[:rows]
    t0 = time.time()
    oracle.free_matvec(media.k1, x[tid], y[tid], x, y, w.q[0], target_ids=tid, workers=workers)
    t_free_rows = time.time() - t0
    ns = 20000
    sl = slice(0, ns)
    t0 = time.time()
    oracle.scattered_matvec(media, x[tid], y[tid], x[sl], y[sl], w.q[0][sl], workers=workers)
    t_scat = time.time() - t0
    per_matvec = t_free_rows * (n / rows) + t_scat * (n / ns) * 2.0
    return {"value": 1.0 / per_matvec, "unit": "matvecs/s", "cores": workers, "kind": "oracle",
            "sample": "%d full free-space target rows (all %d sources) and the Sommerfeld part for "
                      "%d sources x %d targets, extrapolated to one N=%d matvec (%.1f s measured)"
                      % (rows, n, ns, rows, n, t_free_rows + t_scat),
            "seconds_per_matvec_extrapolated": per_matvec}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=1_000_000)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1703_09136_amd as hf
    import workloads

    hf.load()
    dev = torch.device("cuda:0")
    w = workloads.three_layer_ellipses(n=args.n)
    print("workload: %s" % w.name, file=sys.stderr, flush=True)
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    t0 = time.time()
    plan = hf.Plan(w.k, w.interfaces, pts, tol=w.tol, leaf_size=w.leaf)
    torch.cuda.synchronize()
    plan_s = time.time() - t0
    info = plan.info()
    print("plan: %.2f s %s" % (plan_s, json.dumps(info)), file=sys.stderr, flush=True)
    u = torch.empty_like(q)
    for _ in range(args.warmup):
        plan.apply(q, out=u)
    torch.cuda.synchronize()
    print("warmup done", file=sys.stderr, flush=True)

    # timed region: K matvecs, stage events recorded on the same stream
    plan.profile(True)
    plan.profile_read()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        plan.apply(q, out=u)
    end.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    stages, napplies = plan.profile_read()
    plan.profile(False)
    ms = total_ms / args.steps
    stage_avg = {k: v / max(napplies, 1) for k, v in stages.items()}
    print("stage ms per apply: %s" % json.dumps({k: round(v, 4) for k, v in stage_avg.items()}),
          file=sys.stderr, flush=True)

    # accuracy on the oracle's target subset, when the stored values are present
    err = None
    gpath = os.path.join(ROOT, "tests", "golden", "three_layer_oracle.npz")
    if args.n == 1_000_000 and os.path.exists(gpath):
        g = np.load(gpath)
        uu = u.cpu().numpy()[:, g["targets"]]
        err = float(np.linalg.norm(uu - g["u"]) / np.linalg.norm(g["u"]))

    # adjoint seconds
    v = torch.randn_like(q)
    plan.apply_adjoint(v)
    torch.cuda.synchronize()
    a0 = torch.cuda.Event(enable_timing=True)
    a1 = torch.cuda.Event(enable_timing=True)
    a0.record()
    nadj = max(1, args.steps // 4)
    for _ in range(nadj):
        plan.apply_adjoint(v)
    a1.record()
    torch.cuda.synchronize()
    adj_s = a0.elapsed_time(a1) / nadj / 1e3
    # the full backward: A^H v and the source-coordinate gradient
    plan.apply_adjoint(v, q=q, grad_xy=True)
    torch.cuda.synchronize()
    a0.record()
    for _ in range(nadj):
        plan.apply_adjoint(v, q=q, grad_xy=True)
    a1.record()
    torch.cuda.synchronize()
    adj_grad_s = a0.elapsed_time(a1) / nadj / 1e3

    # mixed precision: the near field in FP32, the rest FP64
    plan32 = hf.Plan(w.k, w.interfaces, pts, tol=w.tol, leaf_size=w.leaf, precision=hf.HFMM_FP32)
    for _ in range(args.warmup):
        plan32.apply(q, out=u)
    torch.cuda.synchronize()
    a0.record()
    for _ in range(args.steps):
        plan32.apply(q, out=u)
    a1.record()
    torch.cuda.synchronize()
    ms32 = a0.elapsed_time(a1) / args.steps
    err32 = None
    if args.n == 1_000_000 and os.path.exists(gpath):
        err32 = float(np.linalg.norm(u.cpu().numpy()[:, g["targets"]] - g["u"]) / np.linalg.norm(g["u"]))
    plan32.close()
    mixed = {"precision": "fp32 near field (H0 series, logarithm, per-item sums), fp64 elsewhere",
             "value": 1e3 / ms32, "unit": "matvecs/s", "ms_per_step": ms32, "rel_err_vs_oracle": err32}
    print("mixed: %s" % json.dumps(mixed), file=sys.stderr, flush=True)

    # roofline of the dominant stage
    dominant = max(("m2l", "p2p"), key=lambda s: stage_avg[s])
    if dominant == "m2l":
        work = info["flops_m2l"]
    else:
        # flops of the direct part as the plan evaluates it (series length by
        # item class, logarithm, complex multiply-adds)
        work = info["flops_p2p"]
    dom_s = stage_avg[dominant] / 1e3
    achieved = work / dom_s / 1e12
    roofline = {"bound": "alu", "kernel": dominant, "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                "stage_ms": {k: round(v, 4) for k, v in stage_avg.items()}}

    cpu = None
    if not args.no_cpu_baseline:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline_sample(w)

    out = {"metric": METRIC, "value": 1e3 / ms, "unit": "matvecs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "three-layer k=2pi*(80,120,100), N=%d on 64 ellipses, 1 RHS, tol 1e-8, leaf 64"
                      % w.n, "n": w.n, "nrhs": 1, "tol": w.tol, "leaf": w.leaf,
                      "parallelism": "single GPU"},
           "rel_err_vs_oracle": err, "adjoint_s": adj_s, "adjoint_with_coordinate_grad_s": adj_grad_s,
           "mixed": mixed, "plan_s": plan_s,
           "levels": info["levels"], "orders": info["order"],
           "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
