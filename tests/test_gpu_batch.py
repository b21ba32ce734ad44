"""Batched geometries (hfmm_plan_batch / hfmm_apply_batch), graph replay and
right-hand sides processed in several passes, against single-plan applies of
the same library and the oracle.

Bar: batch results equal the single-plan results to 1e-13 relative (the only
difference is the order of floating-point atomic additions); graph replays
equal eager applies on the same inputs to 1e-13; chunked multi-RHS applies
equal one-pass applies to 1e-13; the oracle bar of the plan tolerance.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
K3S = (2 * np.pi * 20, 2 * np.pi * 30, 2 * np.pi * 25)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _geometries(seed, sizes):
    rng = workloads.rng_for(1703, 9136, seed)
    out = []
    for n in sizes:
        xy = workloads.ellipse_points(rng, n, 8, (0.55, 0.9), 0.51)
        out.append(xy)
    return out


def test_batch_matches_single_plans_and_oracle(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    sizes = [300, 1200, 700, 2000, 90]
    geos = _geometries(91, sizes)
    nrhs = 3
    rng = workloads.rng_for(1703, 9136, 92)
    qs = [workloads.complex_normal(rng, (nrhs, n)) for n in sizes]
    pts = [torch.tensor(xy, dtype=torch.float64, device=dev) for xy in geos]
    qt = [torch.tensor(q, dtype=torch.complex128, device=dev) for q in qs]
    b = gpu_lib.Batch(K3S, (0.5, 0.0), pts, tol=1e-10, leaf_size=32)
    ub = [u.cpu().numpy() for u in b.apply(qt)]
    torch.cuda.synchronize()
    media = oracle.Media(K3S, (0.5, 0.0))
    for g, n in enumerate(sizes):
        p = gpu_lib.Plan(K3S, (0.5, 0.0), pts[g], tol=1e-10, leaf_size=32)
        us = p.apply(qt[g]).cpu().numpy()
        assert rel(ub[g], us) < 1e-13, g
        assert b.info(g)["levels"] == p.info()["levels"]
        p.close()
    g = 1
    ref = oracle.direct_apply(media, geos[g], qs[g])
    e = rel(ub[g], ref)
    print("batch geometry %d E = %.3e" % (g, e))
    assert e < 1e-9
    b.close()


def test_batch_graph_replays_match_eager(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    sizes = [800, 1500, 400]
    geos = _geometries(93, sizes)
    pts = [torch.tensor(xy, dtype=torch.float64, device=dev) for xy in geos]
    b = gpu_lib.Batch(K3S, (0.5, 0.0), pts, tol=1e-8, leaf_size=32)
    singles = [gpu_lib.Plan(K3S, (0.5, 0.0), p, tol=1e-8, leaf_size=32) for p in pts]
    rng = workloads.rng_for(1703, 9136, 94)
    q = [torch.zeros((2, n), dtype=torch.complex128, device=dev) for n in sizes]
    u = [torch.zeros_like(t) for t in q]
    s = torch.cuda.Stream()
    b.graph(True)
    for rep in range(4):
        # eager work between replays: new strengths written into the same buffers
        for t, n in zip(q, sizes):
            t.copy_(torch.tensor(workloads.complex_normal(rng, (2, n)), dtype=torch.complex128, device=dev))
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            b.apply(q, outs=u, stream=s)
        s.synchronize()
        for g in range(len(sizes)):
            ref = singles[g].apply(q[g]).cpu().numpy()
            e = rel(u[g].cpu().numpy(), ref)
            assert e < 1e-13, (rep, g, e)
        torch.cuda.synchronize()
    for p in singles:
        p.close()
    b.close()


def test_rhs_in_several_passes(gpu_lib, monkeypatch):
    import torch
    dev = torch.device("cuda:0")
    w = workloads.two_layer_uniform(n=1024, seed=95, nrhs=7)
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    p = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-10, leaf_size=32)
    u1 = p.apply(q).cpu().numpy()
    v = torch.tensor(workloads.complex_normal(workloads.rng_for(1703, 9136, 96), (7, w.n)), dtype=torch.complex128,
                     device=dev)
    w1, g1 = p.apply_adjoint(v, q=q, grad_xy=True)
    monkeypatch.setenv("HFMM_RHS_CHUNK", "3")
    u3 = p.apply(q).cpu().numpy()
    w3, g3 = p.apply_adjoint(v, q=q, grad_xy=True)
    assert rel(u3, u1) < 1e-13
    assert rel(w3.cpu().numpy(), w1.cpu().numpy()) < 1e-13
    assert rel(g3.cpu().numpy(), g1.cpu().numpy()) < 1e-12
    p.close()
