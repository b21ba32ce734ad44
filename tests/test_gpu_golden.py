"""GPU parity at full size against stored oracle values.

The stored values were written by tests/golden/make_golden.py, which calls only
the oracle: u = A q at a seeded subset of the targets. The inputs are
regenerated from the same seeds. Bar: relative L2 error over the subset below
the plan tolerance 1e-8 (the launch configuration of the benchmark for the
three-layer workload).
"""
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def check(gpu_lib, w, name, tol, **options):
    import torch
    path = os.path.join(HERE, "golden", name + "_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle values %s not generated" % name)
    g = np.load(path)
    dev = torch.device("cuda:0")
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    plan = gpu_lib.Plan(w.k, w.interfaces, pts, tol=tol, leaf_size=w.leaf, **options)
    u = plan.apply(q).cpu().numpy()[:, g["targets"]]
    e = float(np.linalg.norm(u - g["u"]) / np.linalg.norm(g["u"]))
    print(name, "E =", e, plan.info())
    assert e < tol
    return plan


def test_two_layer_high_frequency_n131072(gpu_lib):
    check(gpu_lib, workloads.two_layer_hf(), "two_layer_hf", 1e-8)


@pytest.mark.parametrize("top_level", [0, 2])
def test_three_layer_n1e6(gpu_lib, top_level):
    """top_level 0 is the benchmark's configuration; 2 translates every
    separated pair at its coarsest level."""
    check(gpu_lib, workloads.three_layer_ellipses(), "three_layer", 1e-8, top_level=top_level)
