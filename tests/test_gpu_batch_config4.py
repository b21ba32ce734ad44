"""The batched workload at its own shape: the smallest, a median and the
largest of its 32 three-layer geometries (4478, 16558 and 182595 points)
applied as one batch with 8 right-hand sides, FP64, tolerance 1e-8.

Bars: every geometry of the batch equals a single FP64 plan of the same
geometry to 1e-12 (batching changes only the order of rounding); the largest
geometry agrees with stored oracle values (512 targets, all 8 right-hand
sides, written by tests/golden/make_golden.py) to the tolerance 1e-8.
"""
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
NRHS = 8


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_batched_workload_geometries(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    ids = (workloads.BATCHED_SMALLEST, workloads.BATCHED_MEDIAN, workloads.BATCHED_LARGEST)
    ws = [workloads.batched_geometry(g, nrhs=NRHS) for g in ids]
    pts = [torch.tensor(w.xy, dtype=torch.float64, device=dev) for w in ws]
    qs = [torch.tensor(w.q, dtype=torch.complex128, device=dev) for w in ws]
    b = gpu_lib.Batch(workloads.THREE_LAYER_K, workloads.THREE_LAYER_IF, pts, tol=1e-8, leaf_size=64)
    ub = [u.cpu().numpy() for u in b.apply(qs)]
    for g, w in enumerate(ws):
        p = gpu_lib.Plan(w.k, w.interfaces, pts[g], tol=1e-8, leaf_size=64)
        us = p.apply(qs[g]).cpu().numpy()
        e = rel(ub[g], us)
        print("geometry %d (N=%d): batch vs single plan %.2e" % (ids[g], w.n, e))
        assert e < 1e-12
        p.close()
    path = os.path.join(HERE, "golden", "batched_largest_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle values batched_largest not generated")
    gold = np.load(path)
    e = rel(ub[2][:, gold["targets"]], gold["u"])
    print("largest geometry vs oracle (%d targets x %d rhs): E = %.3e" % (gold["targets"].size, NRHS, e))
    assert e < 1e-8
    b.close()
