"""Mixed precision (HFMM_FP32: the free-space direct pairs in single
precision, everything else FP64) against the oracle.

Bar: relative L2 error below 1e-6 (single-precision pair arithmetic, about
1e-7 expected, on top of the plan tolerance), and the FP32 plan within 1e-6
of the FP64 plan on the same inputs.
"""
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
FP32 = 1


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _apply(hf, w, tol, **opts):
    import torch
    dev = torch.device("cuda:0")
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    plan = hf.Plan(w.k, w.interfaces, pts, tol=tol, **opts)
    return plan, plan.apply(q).cpu().numpy()


def test_fp32_near_field_two_layer_n1024(gpu_lib):
    w = workloads.two_layer_uniform()
    _, u32 = _apply(gpu_lib, w, 1e-10, leaf_size=32, precision=FP32)
    _, u64 = _apply(gpu_lib, w, 1e-10, leaf_size=32)
    ref = oracle.direct_apply(oracle.Media(w.k, w.interfaces), w.xy, w.q)
    e32, e64 = rel(u32, ref), rel(u64, ref)
    print("N=1024 E(fp32) =", e32, "E(fp64) =", e64)
    assert e32 < 1e-6
    assert rel(u32, u64) < 1e-6


def test_fp32_near_field_multiple_rhs_and_adjoint(gpu_lib):
    import torch
    w = workloads.two_layer_uniform(n=900, seed=21, nrhs=3)
    dev = torch.device("cuda:0")
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    plan = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-10, leaf_size=32, precision=FP32)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    u = plan.apply(q).cpu().numpy()
    media = oracle.Media(w.k, w.interfaces)
    ref = oracle.direct_apply(media, w.xy, w.q)
    assert rel(u, ref) < 1e-6
    v = workloads.complex_normal(workloads.rng_for(1703, 9136, 22), (3, w.n))
    wv = plan.apply_adjoint(torch.tensor(v, dtype=torch.complex128, device=dev)).cpu().numpy()
    wref = np.conj(oracle.direct_apply(media, w.xy, np.conj(v)))
    assert rel(wv, wref) < 1e-6


def test_fp32_near_field_three_layer_n1e6(gpu_lib):
    import torch
    path = os.path.join(HERE, "golden", "three_layer_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle values not generated")
    g = np.load(path)
    w = workloads.three_layer_ellipses()
    plan, u = _apply(gpu_lib, w, w.tol, leaf_size=w.leaf, precision=FP32)
    e = rel(u[:, g["targets"]], g["u"])
    print("three-layer N=1e6 E(fp32 near field) =", e)
    assert e < 1e-6
