"""Near-interface quadrature pairs (Section 5: image pairs that stay non-
admissible at the leaves go to direct quadrature of the Sommerfeld integral),
on point sets that hug the interface so that thousands of leaf pairs take
that path: a strip of points between heights 0.002 and 0.062 over the
interface of the two-layer medium k = (8 pi, 12 pi), no interface refinement,
no wavelength bound on the leaves.

Most of these pairs are far apart in x (image admissibility asks for
vertical separation, so bottom-row leaves pair with the whole bottom row):
they go through the tables of G^s(|X|, Y), the neighbours through the
factorised quadrature.

Bars: the plan against the oracle on sampled targets at the plan tolerance
(1e-10) and against the refined plan of the same points (both within 1e-10 of
A, so within 2e-10 of each other); right-hand sides in several groups of the
three-stage evaluation (11 columns) against single-column applies at 1e-13;
the blocked pipeline against the plane pipeline at 1e-12; the adjoint
against conj(A conj(v)) (A is symmetric) at 1e-12; the coordinate gradient of
11 columns against the sum of single-column gradients at 1e-12; a three-layer
strip against the oracle at 1e-10; and the apply time of the unrefined strip
plan within 3x of the refined one (measured 1.6x).
"""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
K2 = (8 * math.pi, 12 * math.pi)
IFS = (0.0,)
OPTS = dict(tol=1e-10, leaf_size=64, leaf_kb=0.0)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def strip(seed, n, nrhs):
    rng = workloads.rng_for(1703, 9136, seed)
    return workloads.uniform_box(rng, n, 0.0, 1.0, 0.002, 0.062), workloads.complex_normal(rng, (nrhs, n))


def test_strip_parity_with_oracle_and_refined_plan(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    xy, q = strip(101, 20000, 1)
    pts, qt = torch.tensor(xy, device=dev), torch.tensor(q, device=dev)
    plan = gpu_lib.Plan(K2, IFS, pts, interface_refine=0, **OPTS)
    inf = plan.info()
    tree = gpu_lib.build_tree(K2, IFS, pts, interface_refine=0, leaf_size=64, leaf_kb=0.0)
    n_iu = len(tree["iu"])
    print("strip N=20000: %d near-interface box pairs, %d point pairs" % (n_iu, inf["interface_pairs"]))
    assert n_iu >= 1000
    u = plan.apply(qt).cpu().numpy()
    plan.close()
    refined = gpu_lib.Plan(K2, IFS, pts, interface_refine=1, **OPTS)
    assert refined.info()["interface_pairs"] == 0
    ur = refined.apply(qt).cpu().numpy()
    refined.close()
    d = rel(u, ur)
    tid = np.arange(7, 20000, 5000)
    eo = rel(u[:, tid], oracle.direct_apply(oracle.Media(K2, IFS), xy, q, targets=tid))
    print("strip: vs refined plan %.2e, vs oracle (%d targets) %.2e" % (d, tid.size, eo))
    assert d < 2e-10
    assert eo < 1e-10


def test_strip_groups_pipelines_adjoint_gradient(gpu_lib, monkeypatch):
    import torch
    dev = torch.device("cuda:0")
    xy, q = strip(102, 3000, 11)
    pts, qt = torch.tensor(xy, device=dev), torch.tensor(q, device=dev)
    plan = gpu_lib.Plan(K2, IFS, pts, interface_refine=0, **OPTS)
    assert plan.info()["interface_pairs"] > 0
    monkeypatch.setenv("HFMM_BLOCKED", "0")
    u = plan.apply(qt).cpu().numpy()
    cols = np.concatenate([plan.apply(qt[r:r + 1]).cpu().numpy() for r in range(11)])
    eg = rel(u, cols)
    monkeypatch.setenv("HFMM_BLOCKED", "1")
    ub = plan.apply(qt).cpu().numpy()
    eb = rel(ub, u)
    monkeypatch.setenv("HFMM_BLOCKED", "0")
    v = qt.conj() * 0.5 + torch.roll(qt, 1, 0)
    w = plan.apply_adjoint(v).cpu().numpy()
    # v.conj() is a lazy view: the binding resolves it before the call
    wd = np.conj(plan.apply(v.conj()).cpu().numpy())
    assert rel(wd, np.conj(plan.apply(torch.conj_physical(v)).cpu().numpy())) < 1e-14
    ea = rel(w, wd)
    _, g = plan.apply_adjoint(v, q=qt, grad_xy=True)
    gsum = sum(plan.apply_adjoint(v[r:r + 1], q=qt[r:r + 1], grad_xy=True)[1].cpu().numpy() for r in range(11))
    egr = rel(g.cpu().numpy(), gsum)
    print("11 columns: groups vs single %.2e, blocked vs plane %.2e, adjoint %.2e, gradient %.2e"
          % (eg, eb, ea, egr))
    assert eg < 1e-13
    assert eb < 1e-12
    assert ea < 1e-12
    assert egr < 1e-12
    plan.close()


def test_three_layer_strip_against_oracle(gpu_lib):
    """Points hugging the top interface of the three-layer medium (wavenumbers
    of the benchmark scaled down): both the quadrature and the tables carry
    the three-layer sigma_1."""
    import torch
    dev = torch.device("cuda:0")
    k3 = (2 * math.pi * 10, 2 * math.pi * 15, 2 * math.pi * 12.5)
    ifs = (0.5, 0.0)
    rng = workloads.rng_for(1703, 9136, 103)
    n = 3000
    xy = workloads.uniform_box(rng, n, 0.0, 1.0, 0.502, 0.54)
    q = workloads.complex_normal(rng, (1, n))
    plan = gpu_lib.Plan(k3, ifs, torch.tensor(xy, device=dev), interface_refine=0, **OPTS)
    inf = plan.info()
    u = plan.apply(torch.tensor(q, device=dev)).cpu().numpy()
    plan.close()
    tid = np.arange(11, n, n // 8)
    eo = rel(u[:, tid], oracle.direct_apply(oracle.Media(k3, ifs), xy, q, targets=tid))
    print("three-layer strip: %d leaf pairs, vs oracle (%d targets) %.2e" % (inf["interface_leaf_pairs"], tid.size, eo))
    assert inf["interface_leaf_pairs"] > 100
    assert eo < 1e-10


def test_unrefined_strip_time_near_refined(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    xy, q = strip(101, 20000, 1)
    pts, qt = torch.tensor(xy, device=dev), torch.tensor(q, device=dev)

    def median_ms(plan):
        plan.apply(qt)
        torch.cuda.synchronize()
        ts = []
        for _ in range(7):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            plan.apply(qt)
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    p0 = gpu_lib.Plan(K2, IFS, pts, interface_refine=0, **OPTS)
    p1 = gpu_lib.Plan(K2, IFS, pts, interface_refine=1, **OPTS)
    t0, t1 = median_ms(p0), median_ms(p1)
    print("strip N=20000: unrefined %.3f ms (%d leaf pairs), refined %.3f ms: %.2fx"
          % (t0, p0.info()["interface_leaf_pairs"], t1, t0 / t1))
    p0.close()
    p1.close()
    assert t0 < 3.0 * t1
