"""Benchmark: heterogeneous-FMM matvecs per second on one MI355X.

Workload: three layers (interfaces y = 0.5 and y = 0; k = 2pi*(80, 120, 100)
top to bottom), N = 10^6 points on 64 random ellipses in the top layer, one
complex128 right-hand side, FP64, tolerance 1e-8, leaf size 64 (seeded
synthetic inputs, see workloads.three_layer_ellipses).

A step is one hfmm_apply (u = A q) with q and u resident in device memory;
the plan (tree, lists, tables) is built before the timed region. Prints one
JSON line. Besides the headline number it reports the mixed-precision plan
(near field in FP32) with its error, the adjoint with and without coordinate
gradients, the batched workload (32 geometries x 256 right-hand sides), the
impedance half-space's scaling, points hugging an interface without
refinement (near-interface pairs), the roofline of the dominant kernel and
the CPU oracle on a bounded sample.
With --gpus other than 1 it exits: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H-FMM matvecs/sec at N=1e6, 3 layers, rel err 1e-8 (FP64) vs mixed; adjoint s"
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector (and FP64 matrix) peak
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector peak
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_p2p_three_layer_n1e6.txt")
# the near-field kernels and the plan code that sizes their work items
KERNEL_SOURCES = ["p2p.hip", "special.hpp", "common.hpp", "h0_cheb.hpp", "log_table.hpp", "hfmm.hip"]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1703_09136_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic():
    """HBM bytes per apply of the near-field kernels from the profiler counters
    recorded in profiles/, or None when missing or taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(kv["p2p_bytes_per_apply"])
    except (KeyError, ValueError):
        return None


def cpu_baseline_sample(w):
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


def timed(torch, fn, reps):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def extras(hf, torch, np, w, plan, pts, q, u, args, golden):
    """Adjoint timings and the mixed-precision plan on the same workload."""
    v = torch.randn_like(q)
    plan.apply_adjoint(v)
    nadj = max(1, args.steps // 4)
    adj_ms = timed(torch, lambda: plan.apply_adjoint(v), nadj)
    plan.apply_adjoint(v, q=q, grad_xy=True)
    adj_grad_ms = timed(torch, lambda: plan.apply_adjoint(v, q=q, grad_xy=True), nadj)
    plan32 = hf.Plan(w.k, w.interfaces, pts, tol=w.tol, leaf_size=w.leaf, precision=hf.HFMM_FP32)
    for _ in range(args.warmup):
        plan32.apply(q, out=u)
    ms32 = timed(torch, lambda: plan32.apply(q, out=u), args.steps)
    err32 = None
    if golden is not None:
        err32 = float(np.linalg.norm(u.cpu().numpy()[:, golden["targets"]] - golden["u"]) /
                      np.linalg.norm(golden["u"]))
    # the FP32 near field's stage time (HIP events, stages in sequence) against
    # the FP32 vector peak, its flops as for the FP64 plan
    plan32.profile(True)
    plan32.profile_read()
    timed(torch, lambda: plan32.apply(q, out=u), args.steps)
    st32, n32 = plan32.profile_read()
    plan32.profile(False)
    info32 = plan32.info()
    plan32.close()
    p2p_s = st32["p2p"] / max(n32, 1) / 1e3
    ach = info32["flops_p2p"] / p2p_s / 1e12
    mixed = {"precision": "fp32 near field (H0 series, logarithm, per-item sums), fp64 elsewhere",
             "value": 1e3 / ms32, "unit": "matvecs/s", "ms_per_step": ms32, "rel_err_vs_oracle": err32,
             "roofline": {"bound": "alu", "kernel": "k_p2p<float> (six series-class launches per apply)",
                          "achieved": ach, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                          "frac": ach / PEAK_FP32_TFLOPS, "near_field_ms": p2p_s * 1e3}}
    return adj_ms / 1e3, adj_grad_ms / 1e3, mixed


PEAKS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}  # dense MFMA TFLOP/s of MI355X


def blocked_work(info):
    """Algorithmic flops of one right-hand side through the blocked pipeline,
    split by the arithmetic of the stage: the multipole-to-local contraction
    (8 (2P+1)^2 per pair), P2M, M2M, L2L and L2P (the plan's count), and the
    direct pairs as complex multiply-adds (8 per ordered pair; each H0 tile
    is evaluated once for all right-hand sides of a block)."""
    return {"m2l": info["flops_m2l"], "updown": info["flops_updown"], "p2p": 8.0 * info["p2p_pairs"]}


def ideal_seconds(work, prec, nrhs):
    """Sum over stages of algorithmic work / peak (the roofline bound): M2L
    and the near field at the peak of their arithmetic, the rest FP64."""
    m2l_peak = PEAKS[prec]
    p2p_peak = PEAKS["f64"] if prec == "f64" else PEAKS["f32"]
    t = 0.0
    for w in work:
        t += (w["m2l"] / m2l_peak + w["updown"] / PEAKS["f64"] + w["p2p"] / p2p_peak) * nrhs / 1e12
    return t


def batched(hf, torch, np, args):
    """32 three-layer geometries, N_g = round(2^U(12,18)), 256 right-hand sides
    each (strengths drawn on the device from a seeded generator; the first 8
    of the largest geometry are the stored oracle case), applied as one batch
    in FP64 (eager and graph replay), FP32 and BF16 (graph replay). Errors:
    the smallest, median and largest geometries against FP64 single plans on
    the same strengths, and the largest against the stored oracle values."""
    import workloads
    dev = torch.device("cuda:0")
    geos = workloads.batched_geometries(nrhs=1)
    pts = [torch.tensor(g.xy, dtype=torch.float64, device=dev) for g in geos]
    ns = [g.n for g in geos]
    nrhs = args.batch_rhs
    gen = torch.Generator(device=dev)
    gen.manual_seed(1703 * 9136 + 4)
    qs = [torch.randn((nrhs, n), dtype=torch.complex128, device=dev, generator=gen) for n in ns]
    check = (workloads.BATCHED_SMALLEST, workloads.BATCHED_MEDIAN, workloads.BATCHED_LARGEST)
    gold = None
    gpath = os.path.join(ROOT, "tests", "golden", "batched_largest_oracle.npz")
    if os.path.exists(gpath) and nrhs >= 8:
        gold = np.load(gpath)
        big = workloads.BATCHED_LARGEST
        qs[big][:8] = torch.tensor(workloads.batched_geometry(big, nrhs=8).q, dtype=torch.complex128, device=dev)
    # FP64 single plans of the checked geometries
    refs = {}
    for g in check:
        p = hf.Plan(workloads.THREE_LAYER_K, workloads.THREE_LAYER_IF, pts[g], tol=1e-8, leaf_size=64)
        refs[g] = p.apply(qs[g]).cpu().numpy()
        p.close()
    us = [torch.empty_like(t) for t in qs]
    s = torch.cuda.Stream()
    out = {"workload": "32 three-layer geometries of 2^U(12,18) points (%d in all), %d right-hand sides each"
                       % (sum(ns), nrhs), "unit": "matvecs/s (geometry x right-hand side)"}
    legs = [("f64", hf.HFMM_FP64, ("eager", "graph")), ("f32", hf.HFMM_FP32, ("graph",)),
            ("bf16", hf.HFMM_BF16, ("graph",))]
    for name, prec, modes in legs:
        t0 = time.time()
        b = hf.Batch(workloads.THREE_LAYER_K, workloads.THREE_LAYER_IF, pts, tol=1e-8, leaf_size=64, precision=prec)
        torch.cuda.synchronize()
        plan_s = time.time() - t0
        work = [blocked_work(b.info(g)) for g in range(len(ns))]
        ms = {}
        for mode in modes:
            b.graph(mode == "graph")
            with torch.cuda.stream(s):
                b.apply(qs, outs=us, stream=s)  # warm-up (graph: capture and first replay)
            s.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            reps = 3
            with torch.cuda.stream(s):
                e0.record(s)
                for _ in range(reps):
                    b.apply(qs, outs=us, stream=s)
                e1.record(s)
            s.synchronize()
            ms[mode] = e0.elapsed_time(e1) / reps
            print("batched %s %s: %.1f ms per batch" % (name, mode, ms[mode]), file=sys.stderr, flush=True)
        errs = {}
        for g in check:
            u = us[g].cpu().numpy()
            errs[str(g)] = float(np.linalg.norm(u - refs[g]) / np.linalg.norm(refs[g]))
        e_or = None
        if gold is not None:
            u = us[workloads.BATCHED_LARGEST][:8].cpu().numpy()[:, gold["targets"]]
            e_or = float(np.linalg.norm(u - gold["u"]) / np.linalg.norm(gold["u"]))
        b.close()
        best = min(ms, key=ms.get)
        t_ideal = ideal_seconds(work, name, nrhs)
        out[name] = {"value": len(ns) * nrhs / ms[best] * 1e3, "ms_per_batch": ms[best], "mode": best,
                     "ms_per_mode": ms, "point_rhs_per_s": sum(ns) * nrhs / ms[best] * 1e3, "plan_s": plan_s,
                     "rel_err_vs_fp64_single_plans": errs, "rel_err_vs_oracle_largest_8rhs": e_or,
                     "roofline": {"bound": "mfma", "ideal_ms": t_ideal * 1e3, "frac": t_ideal * 1e3 / ms[best],
                                  "work_tflop": sum((w["m2l"] + w["updown"] + w["p2p"]) for w in work) * nrhs / 1e12,
                                  "peaks_tflops": {"m2l": PEAKS[name], "near": PEAKS["f64" if name == "f64" else "f32"],
                                                   "other": PEAKS["f64"]}}}
        print("batched %s: %s" % (name, json.dumps(out[name])), file=sys.stderr, flush=True)
    out["value"] = out["f64"]["value"]
    return out


def many_rhs(hf, torch, np, w, pts, golden, args):
    """The N = 10^6 geometry with 64 right-hand sides per apply (the blocked
    pipeline) in FP64, FP32 and BF16: matvecs/s as right-hand sides per
    second, the error of the first right-hand side (the workload's strengths)
    against the stored oracle values and of all against FP64."""
    dev = torch.device("cuda:0")
    nrhs = args.many_rhs
    gen = torch.Generator(device=dev)
    gen.manual_seed(1703 * 9136 + 3)
    q = torch.randn((nrhs, w.n), dtype=torch.complex128, device=dev, generator=gen)
    q[0] = torch.tensor(w.q[0], dtype=torch.complex128, device=dev)
    u = torch.empty_like(q)
    out = {"workload": "three-layer N=%d, %d right-hand sides per apply" % (w.n, nrhs),
           "unit": "matvecs/s (right-hand sides per second)"}
    u64 = None
    for name, prec in (("f64", hf.HFMM_FP64), ("f32", hf.HFMM_FP32), ("bf16", hf.HFMM_BF16)):
        plan = hf.Plan(w.k, w.interfaces, pts, tol=w.tol, leaf_size=w.leaf, precision=prec)
        work = [blocked_work(plan.info())]
        plan.apply(q, out=u)
        torch.cuda.synchronize()
        ms = timed(torch, lambda: plan.apply(q, out=u), max(2, args.steps // 5))
        un = u.cpu().numpy()
        if u64 is None:
            u64 = un
        e_or = None
        if golden is not None:
            e_or = float(np.linalg.norm(un[0:1, golden["targets"]] - golden["u"]) / np.linalg.norm(golden["u"]))
        t_ideal = ideal_seconds(work, name, nrhs)
        out[name] = {"value": nrhs / ms * 1e3, "ms_per_apply": ms, "rel_err_vs_oracle_rhs0": e_or,
                     "rel_err_vs_fp64": float(np.linalg.norm(un - u64) / np.linalg.norm(u64)),
                     "roofline": {"bound": "mfma", "ideal_ms": t_ideal * 1e3, "frac": t_ideal * 1e3 / ms}}
        print("many rhs %s: %s" % (name, json.dumps(out[name])), file=sys.stderr, flush=True)
        plan.close()
    return out


def impedance_scaling(hf, torch, np):
    """The impedance half-space of the paper's numerical results (alpha = 1,
    points on sqrt(N) x sqrt(N) grids in the unit box centred at (0, 1.5),
    p = 39 terms at every level, one right-hand side): milliseconds per apply
    against N, beside the paper's CPU seconds (Table 2, k = 0.1, context only:
    another machine). Measured at k = 1, for which the paper reports the same
    timings; at k = 0.1 the unscaled expansions leave the FP64 range below the
    fourth level, which N > 10^4 needs."""
    import math
    t2 = json.load(open(os.path.join(ROOT, "tests", "golden", "impedance_table2.json")))
    dev = torch.device("cuda:0")
    rows = []
    for n, cpu_s in zip(t2["n"], t2["cpu_seconds"]):
        g = int(round(math.sqrt(n)))
        c = (np.arange(g) + 0.5) / g - 0.5
        X, Y = np.meshgrid(c, c + 1.5)
        pts = torch.tensor(np.stack([X.ravel(), Y.ravel()], 1), dtype=torch.float64, device=dev)
        gen = torch.Generator(device=dev)
        gen.manual_seed(1703 * 9136 + 5)
        q = torch.randn(g * g, dtype=torch.complex128, device=dev, generator=gen)
        plan = hf.Plan((1.0,), (0.0,), pts, tol=1e-10, impedance=1.0, order=39)
        u = plan.apply(q)
        torch.cuda.synchronize()
        ms = timed(torch, lambda: plan.apply(q, out=u), 10)
        rows.append({"n": g * g, "ms_per_apply": ms, "levels": plan.info()["levels"],
                     "paper_cpu_seconds_k0.1": cpu_s})
        plan.close()
    out = {"workload": "impedance half-space alpha=1, k=1, p=39, sqrt(N) grids in the unit box at (0, 1.5)",
           "rows": rows}
    print("impedance: %s" % json.dumps(out), file=sys.stderr, flush=True)
    return out


def near_interface(hf, torch, np):
    """Points hugging the interface without interface refinement: a strip of
    2e4 points between heights 0.002 and 0.062 over the two-layer interface
    (k = 8 pi, 12 pi; leaf 64, no wavelength bound), whose bottom-row leaves
    keep non-admissible image pairs with the whole bottom row. Milliseconds
    per apply of the unrefined plan (near-interface quadrature and tables)
    against the refined plan of the same points, and their difference (both
    within the tolerance 1e-10 of A)."""
    import math
    import workloads
    dev = torch.device("cuda:0")
    rng = workloads.rng_for(1703, 9136, 101)
    xy = workloads.uniform_box(rng, 20000, 0.0, 1.0, 0.002, 0.062)
    pts = torch.tensor(xy, dtype=torch.float64, device=dev)
    k2 = (8 * math.pi, 12 * math.pi)
    res = {}
    for nrhs in (1, 16):
        q = torch.tensor(workloads.complex_normal(rng, (nrhs, xy.shape[0])), dtype=torch.complex128, device=dev)
        row = {}
        u = {}
        for refine in (0, 1):
            plan = hf.Plan(k2, (0.0,), pts, tol=1e-10, leaf_size=64, leaf_kb=0.0, interface_refine=refine)
            u[refine] = plan.apply(q)
            torch.cuda.synchronize()
            inf = plan.info()
            row["refine%d" % refine] = {"ms_per_apply": timed(torch, lambda: plan.apply(q, out=u[refine]), 10),
                                       "interface_leaf_pairs": inf["interface_leaf_pairs"],
                                       "interface_pairs": inf["interface_pairs"]}
            plan.close()
        row["ratio"] = row["refine0"]["ms_per_apply"] / row["refine1"]["ms_per_apply"]
        row["rel_diff"] = float(torch.linalg.norm(u[0] - u[1]) / torch.linalg.norm(u[1]))
        res["nrhs%d" % nrhs] = row
    out = {"workload": "two-layer k=(8pi,12pi), 2e4 points in [0,1]x[0.002,0.062], leaf 64, tol 1e-10, "
                       "interface_refine 0 vs 1", "rows": res}
    print("near-interface: %s" % json.dumps(out), file=sys.stderr, flush=True)
    return out


def cross_layer(hf, torch, np, w, pts, q):
    """Fields below the top interface (hfmm_transmit): the headline workload's
    top-layer points and strengths as sources, 10^5 targets uniform in x over
    [0, 1] and in depth over [0.02, 0.9] below the top interface (the middle
    layer and the bottom one). Milliseconds per call and source-target pairs
    per second; the error against the oracle on a subset (64 sources, 16
    targets, the same call)."""
    import oracle
    import workloads
    dev = torch.device("cuda:0")
    rng = workloads.rng_for(1703, 9136, 301)
    yif = w.interfaces[0]
    tgt = np.c_[rng.uniform(0.0, 1.0, 100_000), yif - rng.uniform(0.02, 0.9, 100_000)]
    tg = torch.tensor(tgt, dtype=torch.float64, device=dev)
    tol = 1e-8
    u = hf.transmit(w.k, w.interfaces, pts, q, tg, tol=tol)
    ms = timed(torch, lambda: hf.transmit(w.k, w.interfaces, pts, q, tg, tol=tol), 3)
    si = rng.choice(pts.shape[0], 64, replace=False)
    ti = rng.choice(tgt.shape[0], 16, replace=False)
    xs, qs = w.xy[si], w.q[:, si]
    us = hf.transmit(w.k, w.interfaces, torch.tensor(xs, device=dev), torch.tensor(qs, device=dev),
                     torch.tensor(tgt[ti], device=dev), tol=tol).cpu().numpy()
    ref = oracle.cross_layer_apply(oracle.Media(w.k, w.interfaces), xs, qs, tgt[ti])
    err = float(np.linalg.norm(us - ref) / np.linalg.norm(ref))
    ns, nt = int(pts.shape[0]), tgt.shape[0]
    # the reverse pairs: the 10^5 points below as sources, the headline points as targets
    qb = torch.tensor(workloads.complex_normal(rng, (1, nt)), dtype=torch.complex128, device=dev)
    uu = hf.transmit(w.k, w.interfaces, tg, qb, pts, tol=tol, up=True)
    ms_up = timed(torch, lambda: hf.transmit(w.k, w.interfaces, tg, qb, pts, tol=tol, up=True), 3)
    out = {"workload": "three-layer k=2pi*(80,120,100): %d top-layer sources (the headline points), %d targets "
                       "at depths 0.02-0.9 below the top interface, tol %g; the reverse pairs with the two sets "
                       "exchanged" % (ns, nt, tol),
           "ms_per_call": ms, "pairs_per_s": ns * nt / ms * 1e3, "rel_err_vs_oracle_subset": err,
           "ms_per_call_reverse": ms_up,
           "finite": bool(torch.isfinite(torch.view_as_real(u)).all() and torch.isfinite(torch.view_as_real(uu)).all())}
    print("cross-layer: %s" % json.dumps(out), file=sys.stderr, flush=True)
    return out


def middle_layer(hf, torch, np):
    """Points in the middle layer (the slab): 10^6 points on 64 ellipses with
    centres uniform in the slab, k = 2 pi (80, 120, 100), tol 1e-8. The matvec
    is the free part (a plan whose layers all have the slab's wavenumber) plus
    the middle layer's scattered part (hfmm_middle_scattered); milliseconds of
    each, and the scattered part's error against the oracle on a 32-point
    subset (its own matvec)."""
    import oracle
    import workloads
    dev = torch.device("cuda:0")
    w = workloads.middle_layer_ellipses()
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    k2 = w.k[1]
    plan = hf.Plan((k2, k2), (float(w.xy[:, 1].min()) - 1.0,), pts, tol=w.tol, leaf_size=w.leaf)
    uf = plan.apply(q)
    ms_free = timed(torch, lambda: plan.apply(q, out=uf), 5)
    plan.close()
    us = hf.middle_scattered(w.k, w.interfaces, pts, q, pts, tol=w.tol)
    ms_scat = timed(torch, lambda: hf.middle_scattered(w.k, w.interfaces, pts, q, pts, tol=w.tol), 2)
    rng = workloads.rng_for(1703, 9136, 303)
    si = rng.choice(w.xy.shape[0], 32, replace=False)
    xs, qs = w.xy[si], w.q[:, si]
    p2 = torch.tensor(xs, device=dev)
    ug = hf.middle_scattered(w.k, w.interfaces, p2, torch.tensor(qs, device=dev), p2, tol=w.tol).cpu().numpy()
    ref = oracle.middle_apply(oracle.Media(w.k, w.interfaces), xs, qs, scattered_only=True)
    err = float(np.linalg.norm(ug - ref) / np.linalg.norm(ref))
    out = {"workload": "three-layer k=2pi*(80,120,100), N=%d on 64 ellipses in the middle layer, tol %g"
                       % (w.xy.shape[0], w.tol),
           "ms_free_part": ms_free, "ms_scattered_part": ms_scat, "ms_per_matvec": ms_free + ms_scat,
           "matvecs_per_s": 1e3 / (ms_free + ms_scat), "rel_err_scattered_vs_oracle_subset": err,
           "finite": bool(torch.isfinite(torch.view_as_real(us)).all())}
    print("middle layer: %s" % json.dumps(out), file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=30,
                    help="untimed applies first (the GPU reaches its steady clocks within a few dozen)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the adjoint, mixed-precision and batched legs (profiling runs)")
    ap.add_argument("--batch-rhs", type=int, default=256)
    ap.add_argument("--many-rhs", type=int, default=64)
    ap.add_argument("--legs", default="adjoint,mixed,many,batched,impedance,iface,xlayer,middle",
                    help="side legs to run besides the headline (profiling runs pick one)")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--leaf", type=int, default=0, help="points per leaf (0: the workload's)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1703_09136_amd as hf
    import workloads

    hf.load()
    dev = torch.device("cuda:0")
    w = workloads.three_layer_ellipses(n=args.n)
    if args.leaf > 0:
        w.leaf = args.leaf
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
    # a plain copy of known size (16 B per point each way): it calibrates the
    # HBM byte counters of the profiler runs
    q.clone()
    for _ in range(args.warmup):
        plan.apply(q, out=u)
    torch.cuda.synchronize()
    print("warmup done", file=sys.stderr, flush=True)

    # timed region: K matvecs as a caller runs them (the near field on the
    # plan's side stream beside the far-field chain)
    ms = timed(torch, lambda: plan.apply(q, out=u), args.steps)
    # stage durations: the same matvecs with HIP events between the stages,
    # which then run one after another on the apply stream
    plan.profile(True)
    plan.profile_read()
    ms_serial = timed(torch, lambda: plan.apply(q, out=u), args.steps)
    stages, napplies = plan.profile_read()
    plan.profile(False)
    stage_avg = {k: v / max(napplies, 1) for k, v in stages.items()}
    print("stage ms per apply: %s" % json.dumps({k: round(v, 4) for k, v in stage_avg.items()}),
          file=sys.stderr, flush=True)

    # accuracy on the oracle's target subset, when the stored values are present
    err = None
    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", "three_layer_oracle.npz")
    if args.n == 1_000_000 and os.path.exists(gpath):
        golden = np.load(gpath)
        err = float(np.linalg.norm(u.cpu().numpy()[:, golden["targets"]] - golden["u"]) /
                    np.linalg.norm(golden["u"]))

    # roofline of the dominant stage (the near field or M2L), its time from the
    # HIP events recorded on the apply stream around its launches
    dominant = max(("m2l", "p2p"), key=lambda k: stage_avg[k])
    if dominant == "m2l":
        work = info["flops_m2l"]
        kname = "k_trans_mfma + k_reduce_contrib (M2L)"
        traffic = None
    else:
        # flops of the direct part as the plan evaluates it (series length by
        # item class, logarithm, complex multiply-adds)
        work = info["flops_p2p"]
        kname = "k_p2p (six series-class launches per apply)"
        traffic = stored_traffic()
    dom_s = stage_avg[dominant] / 1e3
    achieved = work / dom_s / 1e12
    roofline = {"bound": "alu", "kernel": kname, "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                "stage_ms": {k: round(v, 4) for k, v in stage_avg.items()},
                "ms_per_step_stages_in_sequence": ms_serial}

    adj_s = adj_grad_s = mixed = batch = many = imp = None
    legs = set() if args.no_extras else set(args.legs.split(","))
    if legs & {"adjoint", "mixed"}:
        adj_s, adj_grad_s, mixed = extras(hf, torch, np, w, plan, pts, q, u, args, golden)
        print("mixed: %s" % json.dumps(mixed), file=sys.stderr, flush=True)
    imp = impedance_scaling(hf, torch, np) if "impedance" in legs else None
    iface = near_interface(hf, torch, np) if "iface" in legs else None
    xlayer = cross_layer(hf, torch, np, w, pts, q) if "xlayer" in legs else None
    middle = middle_layer(hf, torch, np) if "middle" in legs else None
    if "many" in legs:
        many = many_rhs(hf, torch, np, w, pts, golden, args)
    if "batched" in legs:
        batch = batched(hf, torch, np, args)
    plan.close()

    cpu = None
    if not args.no_cpu_baseline:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline_sample(w)

    out = {"metric": METRIC, "value": 1e3 / ms, "unit": "matvecs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "three-layer k=2pi*(80,120,100), N=%d on 64 ellipses, 1 RHS, tol 1e-8, leaf %d"
                      % (w.n, w.leaf), "n": w.n, "nrhs": 1, "tol": w.tol, "leaf": w.leaf,
                      "parallelism": "single GPU"},
           "rel_err_vs_oracle": err, "adjoint_s": adj_s, "adjoint_with_coordinate_grad_s": adj_grad_s,
           "mixed": mixed, "many_rhs": many, "batched": batch, "impedance": imp, "near_interface": iface, "cross_layer": xlayer, "middle_layer": middle, "plan_s": plan_s,
           "levels": info["levels"], "orders": info["order"],
           "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
