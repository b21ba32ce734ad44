"""GPU parity: the HIP library (through the C interface) against the CPU oracle.

Bar: relative L2 error E = ||u - u_ref|| / ||u_ref|| over all targets and
right-hand sides, below the plan tolerance (1e-10 for the two-layer workload
at N = 1024, 1e-8 otherwise); 1e-12 where every pair is evaluated directly.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

K3S = (2 * math.pi * 20, 2 * math.pi * 30, 2 * math.pi * 25)   # three-layer medium, reduced frequency


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run(hf, w, tol, q=None, **opts):
    import torch
    dev = torch.device("cuda:0")
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    qq = torch.tensor(w.q if q is None else q, dtype=torch.complex128, device=dev)
    plan = hf.Plan(w.k, w.interfaces, pts, tol=tol, **opts)
    u = plan.apply(qq).cpu().numpy()
    return plan, u


def ref_apply(w, q=None):
    return oracle.direct_apply(oracle.Media(w.k, w.interfaces), w.xy, w.q if q is None else q)


def test_one_leaf_plan_is_the_direct_sum(gpu_lib):
    """Every pair direct: free H0 pairs plus Sommerfeld quadrature of the image."""
    w = workloads.two_layer_uniform(n=200, seed=11)
    plan, u = run(gpu_lib, w, 1e-10, leaf_size=256, interface_refine=0, leaf_kb=0.0)
    assert plan.info()["levels"] == 1
    e = rel(u, ref_apply(w))
    print("one-leaf E =", e)
    assert e < 1e-12


@pytest.mark.parametrize("top_level", [0, 2, 3])
def test_two_layer_n1024_full_tree(gpu_lib, top_level):
    """top_level 2: every separated pair at its coarsest level (M2M and L2L on
    every level); 0: the automatic top level; 3: in between."""
    w = workloads.two_layer_uniform()
    plan, u = run(gpu_lib, w, 1e-10, leaf_size=32, top_level=top_level)
    inf = plan.info()
    e = rel(u, ref_apply(w))
    print("two-layer N=1024 top_level %d E =" % top_level, e, inf)
    assert inf["m2l_pairs"] > 0 and inf["image_pairs"] > 0
    if top_level:
        assert inf["top_level"] == top_level
    assert e < 1e-10


def test_two_layer_without_interface_refinement(gpu_lib):
    """Image pairs left non-admissible at the leaves go to direct quadrature."""
    w = workloads.two_layer_uniform(n=1024, seed=12)
    plan, u = run(gpu_lib, w, 1e-10, leaf_size=32, interface_refine=0, leaf_kb=0.0)
    inf = plan.info()
    e = rel(u, ref_apply(w))
    print("no-refine E =", e, inf)
    assert inf["interface_pairs"] > 0
    assert e < 1e-10


def test_three_layer_reduced_frequency(gpu_lib):
    rng = workloads.rng_for(1703, 9136, 33)
    xy = workloads.ellipse_points(rng, 3000, 16, (0.5, 1.0), 0.51)
    q = workloads.complex_normal(rng, (1, xy.shape[0]))
    w = workloads.Workload("three-layer small", K3S, (0.5, 0.0), xy, q, leaf=64, tol=1e-8)
    plan, u = run(gpu_lib, w, 1e-8, leaf_size=64)
    e = rel(u, ref_apply(w))
    print("three-layer small E =", e, plan.info())
    assert e < 1e-8


def test_homogeneous_medium_has_no_scattered_part(gpu_lib):
    w = workloads.two_layer_uniform(n=800, seed=13)
    w.k = (w.k[0], w.k[0])
    plan, u = run(gpu_lib, w, 1e-10, leaf_size=32)
    e = rel(u, ref_apply(w))
    print("homogeneous E =", e)
    assert e < 1e-10


def test_multiple_right_hand_sides(gpu_lib):
    w = workloads.two_layer_uniform(n=600, seed=14, nrhs=3)
    plan, u = run(gpu_lib, w, 1e-10, leaf_size=32)
    e = rel(u, ref_apply(w))
    assert e < 1e-10
    import torch
    for r in range(3):
        q1 = torch.tensor(w.q[r], dtype=torch.complex128, device="cuda:0")
        u1 = plan.apply(q1).cpu().numpy()
        assert np.max(np.abs(u1 - u[r])) <= 1e-13 * np.max(np.abs(u[r]))


def test_adjoint_is_the_transpose(gpu_lib):
    import torch
    w = workloads.two_layer_uniform(n=1024, seed=15, nrhs=2)
    plan, u = run(gpu_lib, w, 1e-10, leaf_size=32)
    rng = np.random.default_rng(5)
    v = rng.standard_normal((2, w.n)) + 1j * rng.standard_normal((2, w.n))
    wv = plan.apply_adjoint(torch.tensor(v, dtype=torch.complex128, device="cuda:0")).cpu().numpy()
    lhs = np.vdot(v, u)             # <v, A q>
    rhs = np.vdot(wv, w.q)          # <A^H v, q>
    print("dot test", abs(lhs - rhs) / abs(lhs))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    ref = np.conj(ref_apply(w, np.conj(v)))   # A symmetric: A^H v = conj(A conj v)
    assert rel(wv, ref) < 1e-10


def test_stages_in_sequence_match_overlapped(gpu_lib):
    """Under stage timing the stages run one after another, the form graph
    capture also uses (small M2M levels then gather a child quadrant per wave,
    and the adjoint's small L2L^T levels likewise); forward and adjoint agree
    with the overlapped applies up to the order of rounding."""
    import torch
    w = workloads.three_layer_ellipses(n=20000, seed=17, nrhs=2)
    plan, u = run(gpu_lib, w, 1e-8, leaf_size=64)
    q = torch.tensor(w.q, dtype=torch.complex128, device="cuda:0")
    v = torch.tensor(workloads.complex_normal(workloads.rng_for(1703, 9136, 18), (2, w.n)),
                     dtype=torch.complex128, device="cuda:0")
    wv = plan.apply_adjoint(v).cpu().numpy()
    plan.profile(True)
    us = plan.apply(q).cpu().numpy()
    ws = plan.apply_adjoint(v).cpu().numpy()
    st, napplies = plan.profile_read()
    plan.profile(False)
    print("levels", plan.info()["levels"], "orders", plan.info()["order"], "stages ms", st)
    assert napplies == 1 and st["m2m"] > 0
    assert rel(us, u) < 1e-13
    assert rel(ws, wv) < 1e-13
    plan.close()


def test_tiny_leaves_many_per_wave(gpu_lib):
    """Leaves of a few points: the per-point L2P then finds more than four
    leaves in most 64-point waves and stages them four at a time; forward
    against the oracle, adjoint by the dot test."""
    import torch
    w = workloads.two_layer_uniform(n=1024, seed=19, nrhs=1)
    plan, u = run(gpu_lib, w, 1e-10, leaf_size=4)
    inf = plan.info()
    print("tiny leaves:", inf)
    assert inf["leaves"] > w.n / 8 and inf["m2l_pairs"] > 0
    e = rel(u, ref_apply(w))
    print("tiny-leaf E =", e)
    assert e < 1e-10
    rng = workloads.rng_for(1703, 9136, 20)
    v = workloads.complex_normal(rng, (w.n,))
    wv = plan.apply_adjoint(torch.tensor(v, dtype=torch.complex128, device="cuda:0")).cpu().numpy()
    lhs = np.vdot(v, u.reshape(-1))
    rhs = np.vdot(wv, w.q.reshape(-1))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    plan.close()
