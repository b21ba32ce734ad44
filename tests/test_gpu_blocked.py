"""The right-hand-side-blocked pipeline (many right-hand sides: every stage a
contraction over 64 right-hand sides per block on the matrix cores) against
the plane pipeline of the same plan, the oracle and FP64.

Bars: FP64 blocked vs plane applies of the same plan 1e-12 (both compute the
same FP64 approximation; only the order of rounding differs); blocked vs the
oracle at the plan tolerance; several passes (pass width capped) equal one
pass to 1e-13; FP32 multipole-to-local and near field within 1e-6 of FP64
(the batched workload's bar); BF16 multipole-to-local within 1e-2 of FP64
(its 8-bit mantissa: the measured value is printed).
"""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
K3S = (2 * math.pi * 20, 2 * math.pi * 30, 2 * math.pi * 25)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _apply(hf, plan, q, monkeypatch, blocked):
    monkeypatch.setenv("HFMM_BLOCKED", "1" if blocked else "0")
    u = plan.apply(q).cpu().numpy()
    monkeypatch.delenv("HFMM_BLOCKED")
    return u


def test_blocked_two_layer_against_plane_and_oracle(gpu_lib, monkeypatch):
    import torch
    dev = torch.device("cuda:0")
    w = workloads.two_layer_uniform(n=1024, seed=41, nrhs=64)
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    plan = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-10, leaf_size=32)
    ub = _apply(gpu_lib, plan, q, monkeypatch, True)
    up = _apply(gpu_lib, plan, q, monkeypatch, False)
    e = rel(ub, up)
    print("two-layer N=1024, 64 rhs: blocked vs plane %.2e" % e)
    assert e < 1e-12
    ref = oracle.direct_apply(oracle.Media(w.k, w.interfaces), w.xy, w.q[:4])
    eo = rel(ub[:4], ref)
    print("  blocked vs oracle (4 rhs) %.2e" % eo)
    assert eo < 1e-10
    plan.close()


@pytest.mark.parametrize("top_level", [0, 2])
def test_blocked_three_layer_against_plane(gpu_lib, monkeypatch, top_level):
    import torch
    dev = torch.device("cuda:0")
    rng = workloads.rng_for(1703, 9136, 42)
    xy = workloads.ellipse_points(rng, 3000, 8, (0.55, 0.9), 0.51)
    q = torch.tensor(workloads.complex_normal(rng, (70, 3000)), dtype=torch.complex128, device=dev)
    pts = torch.tensor(xy, dtype=torch.float64, device=dev)
    plan = gpu_lib.Plan(K3S, (0.5, 0.0), pts, tol=1e-10, leaf_size=32, top_level=top_level)
    ub = _apply(gpu_lib, plan, q, monkeypatch, True)
    up = _apply(gpu_lib, plan, q, monkeypatch, False)
    e = rel(ub, up)
    print("three-layer N=3000 top %d, 70 rhs: blocked vs plane %.2e" % (top_level, e))
    assert e < 1e-12
    ref = oracle.direct_apply(oracle.Media(K3S, (0.5, 0.0)), xy, q[:2].cpu().numpy())
    assert rel(ub[:2], ref) < 1e-10
    plan.close()


def test_blocked_several_passes_and_self_none(gpu_lib, monkeypatch):
    import torch
    dev = torch.device("cuda:0")
    w = workloads.two_layer_uniform(n=2000, seed=43, nrhs=130)
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    plan = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-8, leaf_size=32, self_term=gpu_lib.HFMM_SELF_NONE)
    u1 = _apply(gpu_lib, plan, q, monkeypatch, True)
    monkeypatch.setenv("HFMM_BLK_RHS", "64")
    u3 = _apply(gpu_lib, plan, q, monkeypatch, True)
    monkeypatch.delenv("HFMM_BLK_RHS")
    assert rel(u3, u1) < 1e-13
    up = _apply(gpu_lib, plan, q, monkeypatch, False)
    assert rel(u1, up) < 1e-12
    ref = oracle.direct_apply(oracle.Media(w.k, w.interfaces), w.xy, w.q[129:130], self_term=False)
    assert rel(u1[129:130], ref) < 1e-8
    plan.close()


@pytest.mark.parametrize("prec,bar", [("HFMM_FP32", 1e-6), ("HFMM_BF16", 1e-2)])
def test_blocked_reduced_precision_batched_geometries(gpu_lib, prec, bar):
    """The batched workload's smallest and median geometries, 64 right-hand
    sides: reduced-precision plans against the FP64 plan."""
    import torch
    dev = torch.device("cuda:0")
    for g in (workloads.BATCHED_SMALLEST, workloads.BATCHED_MEDIAN):
        w = workloads.batched_geometry(g, nrhs=64)
        pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
        q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
        p64 = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-8, leaf_size=64)
        plo = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-8, leaf_size=64, precision=getattr(gpu_lib, prec))
        u64 = p64.apply(q).cpu().numpy()
        ulo = plo.apply(q).cpu().numpy()
        e = rel(ulo, u64)
        print("%s geometry %d (N=%d): vs FP64 %.3e" % (prec, g, w.n, e))
        assert e < bar
        p64.close()
        plo.close()


def test_blocked_batch_graph_replays(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    rng = workloads.rng_for(1703, 9136, 44)
    sizes = [900, 2500]
    geos = [workloads.ellipse_points(rng, n, 8, (0.55, 0.9), 0.51) for n in sizes]
    pts = [torch.tensor(xy, dtype=torch.float64, device=dev) for xy in geos]
    b = gpu_lib.Batch(K3S, (0.5, 0.0), pts, tol=1e-8, leaf_size=32)
    singles = [gpu_lib.Plan(K3S, (0.5, 0.0), p, tol=1e-8, leaf_size=32) for p in pts]
    q = [torch.zeros((64, n), dtype=torch.complex128, device=dev) for n in sizes]
    u = [torch.zeros_like(t) for t in q]
    s = torch.cuda.Stream()
    b.graph(True)
    for rep in range(3):
        for t, n in zip(q, sizes):
            t.copy_(torch.tensor(workloads.complex_normal(rng, (64, n)), dtype=torch.complex128, device=dev))
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            b.apply(q, outs=u, stream=s)
        s.synchronize()
        for g in range(2):
            e = rel(u[g].cpu().numpy(), singles[g].apply(q[g]).cpu().numpy())
            assert e < 1e-13, (rep, g, e)
    b.close()
    for p in singles:
        p.close()
