"""The C interface on the GPU: domain errors, the self-term option, caller
allocators, reserved workspaces, fixed expansion orders, output checks and
the life of temporaries in the binding.

Bars: domain errors are reported as HFMM_ERR_DOMAIN with no plan returned;
HFMM_SELF_NONE results match the oracle's A with A_ii = 0 at the plan
tolerance (apply, adjoint) and 1e-7 (coordinate gradient, tol 1e-10); the
caller-allocator and reserved-workspace plans equal the default plan to
1e-13 (only the order of atomic additions differs).
"""
import ctypes
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _plan_raw(hf, xy, k=(8 * math.pi, 12 * math.pi), ifs=(0.0,), tol=1e-8, **opts):
    """hfmm_plan through ctypes on device points; returns (status, handle, message)."""
    import torch
    lib = hf.load()
    pts = torch.tensor(np.asarray(xy, float), dtype=torch.float64, device="cuda:0").contiguous()
    h = ctypes.c_void_p()
    kk = (ctypes.c_double * len(k))(*k)
    ii = (ctypes.c_double * len(ifs))(*ifs)
    o = hf.default_options(**opts)
    st = lib.hfmm_plan(ctypes.byref(h), len(k), kk, ii, pts.shape[0], ctypes.c_void_p(pts.data_ptr()), tol,
                       ctypes.byref(o), None)
    torch.cuda.synchronize()
    return st, h, lib.hfmm_last_error_message().decode()


def _points(n=64, seed=31):
    rng = workloads.rng_for(1703, 9136, seed)
    return workloads.uniform_box(rng, n, 0.0, 1.0, 0.05, 1.05)


@pytest.mark.parametrize("case", ["below", "on", "nan", "inf", "coincident", "coincident_apart"])
def test_domain_errors(gpu_lib, case):
    xy = _points()
    if case == "below":
        xy[17, 1] = -0.01
    elif case == "on":
        xy[5, 1] = 0.0
    elif case == "nan":
        xy[9, 0] = float("nan")
    elif case == "inf":
        xy[9, 1] = float("inf")
    elif case == "coincident":
        xy[40] = xy[3]
    elif case == "coincident_apart":
        # two equal points and, between them in index order, a different point
        # whose 60-bit Morton key is the same (it differs by far less than the
        # key resolution)
        base = xy[10].copy()
        xy[20] = base + np.array([1e-13, 0.0])
        xy[30] = base
    st, h, msg = _plan_raw(gpu_lib, xy)
    print(case, st, msg)
    assert st == 2, msg
    assert not h.value
    assert msg


def test_nearly_coincident_points_are_accepted(gpu_lib):
    xy = _points()
    xy[20] = xy[10] + np.array([1e-9, 0.0])
    st, h, msg = _plan_raw(gpu_lib, xy)
    assert st == 0, msg
    gpu_lib.load().hfmm_destroy(h)


def test_self_term_none_apply_adjoint_gradient(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    w = workloads.two_layer_uniform(n=1024, seed=33, nrhs=2)
    media = oracle.Media(w.k, w.interfaces)
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    plan = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-10, leaf_size=32, self_term=gpu_lib.HFMM_SELF_NONE)
    u = plan.apply(q).cpu().numpy()
    ref = oracle.direct_apply(media, w.xy, w.q, self_term=False)
    e = rel(u, ref)
    print("SELF_NONE apply E =", e)
    assert e < 1e-10
    # the difference to the default plan is the scattered self term
    full = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-10, leaf_size=32).apply(q).cpu().numpy()
    yf = media.to_frame(w.xy[:, 1])
    gs = oracle.scattered_pairs(media, np.zeros(w.n), 2 * yf)
    assert rel(full - u, gs[None, :] * w.q) < 1e-9
    v = workloads.complex_normal(workloads.rng_for(1703, 9136, 34), (2, w.n))
    vt = torch.tensor(v, dtype=torch.complex128, device=dev)
    wv, g = plan.apply_adjoint(vt, q=q, grad_xy=True)
    wref = np.conj(oracle.direct_apply(media, w.xy, np.conj(v), self_term=False))
    assert rel(wv.cpu().numpy(), wref) < 1e-10
    gref = oracle.source_gradient(media, w.xy, w.q, v, self_term=False)
    eg = rel(g.cpu().numpy(), gref)
    print("SELF_NONE gradient E =", eg)
    assert eg < 1e-7


def test_caller_allocator_and_reserved_workspace(gpu_lib):
    """torch's caching allocator behind the plan (the binding's default) and
    hipMalloc give the same results; a plan with max_nrhs reserves its
    workspace when it is built."""
    import torch
    dev = torch.device("cuda:0")
    w = workloads.two_layer_uniform(n=2000, seed=35, nrhs=3)
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(dev)
    p_t = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-10, leaf_size=32, torch_allocator=True)
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated(dev) - before
    print("plan memory from torch's allocator: %d bytes" % held)
    assert held > 0
    p_h = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-10, leaf_size=32, torch_allocator=False)
    u_t = p_t.apply(q).cpu().numpy()
    u_h = p_h.apply(q).cpu().numpy()
    assert rel(u_t, u_h) < 1e-13
    p_t.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(dev) - before < held
    p_r = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-10, leaf_size=32, max_nrhs=3)
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated(dev)
    u_r = p_r.apply(q).cpu().numpy()
    torch.cuda.synchronize()
    # nothing but the output tensor is allocated by the apply
    assert torch.cuda.memory_allocated(dev) - m0 <= q.numel() * 16
    assert rel(u_r, u_h) < 1e-13
    p_h.close()
    p_r.close()


def test_fixed_order(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    w = workloads.two_layer_uniform(n=1024, seed=36)
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    ref = oracle.direct_apply(oracle.Media(w.k, w.interfaces), w.xy, w.q)
    errs = []
    for p in (10, 20, 40):
        plan = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-10, leaf_size=32, order=p)
        inf = plan.info()
        assert all(o == p for o in inf["order"][2:])
        errs.append(rel(plan.apply(q).cpu().numpy(), ref))
        plan.close()
    print("fixed orders 10/20/40: E =", errs)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-10


def test_output_checks_and_noncontiguous_strengths(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    w = workloads.two_layer_uniform(n=600, seed=37, nrhs=2)
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    plan = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-10, leaf_size=32)
    with pytest.raises(ValueError):
        plan.apply(q, out=torch.empty((2, w.n - 1), dtype=torch.complex128, device=dev))
    with pytest.raises(TypeError):
        plan.apply(q, out=torch.empty((2, w.n), dtype=torch.complex64, device=dev))
    with pytest.raises(ValueError):
        plan.apply(q, out=q)
    # a non-contiguous q (a column slice) through the adjoint's gradient
    big = torch.zeros((w.n, 4), dtype=torch.complex128, device=dev)
    big[:, 1] = q[0]
    qn = big[:, 1]
    assert not qn.is_contiguous()
    v = torch.tensor(workloads.complex_normal(workloads.rng_for(1703, 9136, 38), (1, w.n)),
                     dtype=torch.complex128, device=dev)
    _, g1 = plan.apply_adjoint(v, q=qn, grad_xy=True)
    _, g2 = plan.apply_adjoint(v, q=q[0:1].contiguous(), grad_xy=True)
    assert rel(g1.cpu().numpy(), g2.cpu().numpy()) < 1e-13
    # the same through autograd with a non-contiguous saved q
    ptsg = pts.clone().requires_grad_(True)
    qa = big[:, 1].clone().requires_grad_(False)
    qs = torch.zeros((w.n, 3), dtype=torch.complex128, device=dev)
    qs[:, 2] = qa
    qv = qs[:, 2].requires_grad_(True)
    u = gpu_lib.hfmm_apply_autograd(qv, plan, ptsg)
    (u.abs() ** 2).sum().backward()
    _, gref = plan.apply_adjoint(2 * u.detach(), q=q[0:1].contiguous(), grad_xy=True)
    assert rel(ptsg.grad.cpu().numpy(), gref.cpu().numpy()) < 1e-12
    plan.close()


def test_batch_graph_after_workspace_growth(gpu_lib):
    """A direct apply with more right-hand sides on a batch's plan grows its
    workspace; the batch's next apply must capture a new graph instead of
    replaying one that points at the released buffers."""
    import torch
    dev = torch.device("cuda:0")
    k3 = (2 * math.pi * 20, 2 * math.pi * 30, 2 * math.pi * 25)
    rng = workloads.rng_for(1703, 9136, 39)
    geos = [workloads.ellipse_points(rng, n, 8, (0.55, 0.9), 0.51) for n in (700, 1300)]
    pts = [torch.tensor(xy, dtype=torch.float64, device=dev) for xy in geos]
    b = gpu_lib.Batch(k3, (0.5, 0.0), pts, tol=1e-8, leaf_size=32)
    singles = [gpu_lib.Plan(k3, (0.5, 0.0), p, tol=1e-8, leaf_size=32) for p in pts]
    q = [torch.tensor(workloads.complex_normal(rng, (1, n)), dtype=torch.complex128, device=dev) for n in (700, 1300)]
    u = [torch.zeros_like(t) for t in q]
    s = torch.cuda.Stream()
    b.graph(True)
    lib = gpu_lib.load()
    for rep in range(3):
        with torch.cuda.stream(s):
            b.apply(q, outs=u, stream=s)
        s.synchronize()
        for g in range(2):
            assert rel(u[g].cpu().numpy(), singles[g].apply(q[g]).cpu().numpy()) < 1e-13, (rep, g)
        # grow plan 1's workspace through the C interface
        h = ctypes.c_void_p()
        assert lib.hfmm_batch_plan(b._h, 1, ctypes.byref(h)) == 0
        qq = torch.tensor(workloads.complex_normal(rng, (2 + 3 * rep, 1300)), dtype=torch.complex128, device=dev)
        uu = torch.empty_like(qq)
        assert lib.hfmm_apply(h, ctypes.c_void_p(qq.data_ptr()), ctypes.c_void_p(uu.data_ptr()), qq.shape[0],
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)) == 0
        torch.cuda.synchronize()
        assert rel(uu.cpu().numpy(), singles[1].apply(qq).cpu().numpy()) < 1e-13
    b.close()
    for p in singles:
        p.close()
